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
#include <type_traits>

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
                                                      int lt, R diag, R c, R c2, cpx<R>* __restrict__ xacc,
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
  } else if (MODE == 1 || MODE == 3) {
    const cpx<R> v0 = x[i0], v1 = x[i1];
    xacc[i0] = MODE == 3 ? c * v0 : xacc[i0] + c * v0;
    xacc[i1] = MODE == 3 ? c * v1 : xacc[i1] + c * v1;
    y[i0] = v0 - c * o0;
    y[i1] = v1 - c * o1;
  } else if (MODE == 4 || MODE == 5) {
    const cpx<R> v0 = x[i0], v1 = x[i1];
    const cpx<R> a0 = MODE == 5 ? c * v0 : xacc[i0] + c * v0;
    const cpx<R> a1 = MODE == 5 ? c * v1 : xacc[i1] + c * v1;
    xacc[i0] = a0 + c2 * (v0 - c * o0);
    xacc[i1] = a1 + c2 * (v1 - c * o1);
  } else {
    y[i0] = aux[i0] - o0;
    y[i1] = aux[i1] - o1;
  }
}

// ---------------------------------------------------------------------------
// Fused A = D^H D (one pass over memory).
//
// A workgroup owns a TX x TT tile.  psi on the tile plus a one-site halo (corners
// included) is staged in LDS.  Phase 1 computes phi = D psi on the tile and, on the
// halo ring, only the spin projection that D^H will use there: for the ring site
// beyond the tile in direction +mu, D^H needs (1 + gamma_mu) phi, which annihilates
// the (1 - gamma_mu) hop of D from that site further out, so that hop (the only
// one reaching past the halo) is skipped.  Phase 2 applies D^H on the tile.  Each
// thread keeps its sites' links and phi in registers between the phases, so the
// algorithmic traffic is psi in + links + y out per site.
//
// Tiles are ordered so that the workgroups that land on one XCD (dispatch is
// round-robin over the 8 XCDs) cover a contiguous band of the lattice; the halos
// they share then hit the same L2.
// ---------------------------------------------------------------------------
// Hop directions for the skip argument.
enum { kSkipNone = -1, kSkipXp = 0, kSkipXm = 1, kSkipTp = 2, kSkipTm = 3 };

template <typename R, bool DAG>
__device__ inline void hop_acc(cpx<R>& s0, cpx<R>& s1, int dir, cpx<R> u, cpx<R> p0, cpx<R> p1) {
  // dir 0: +x (1 -+ s1), 1: -x (1 +- s1), 2: +t (1 -+ s2), 3: -t (1 +- s2); upper sign for D.
  const bool minus = ((dir & 1) == 0) != DAG;  // projector (1 - gamma) ?
  if (dir < 2) {
    if (minus) { cpx<R> h = u * (p0 - p1); s0 = s0 + h; s1 = s1 - h; }
    else       { cpx<R> h = u * (p0 + p1); s0 = s0 + h; s1 = s1 + h; }
  } else {
    if (minus) { cpx<R> h = u * (p0 + imul(p1)); s0 = s0 + h; s1 = s1 - imul(h); }
    else       { cpx<R> h = u * (p0 - imul(p1)); s0 = s0 + h; s1 = s1 + imul(h); }
  }
}

__device__ inline int fused_tile(int b, int nb) {
  // XCD-aware order: block b runs on XCD b % 8; give XCD k the k-th eighth of the tiles.
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// MODE 6 is the CG step of the outer solve: the staged vector is p = z + beta p_old
// (z = x, p_old = aux, beta per right-hand side; p = z where beta = 0), p is written to
// xacc, y = A p, and the workgroup's share of <p, A p> goes to partial[rhs][block].
// MODE 7 ends a V-cycle: the last two smoother steps of MODE 4 (xacc becomes the
// V-cycle's output z) and the workgroup's share of <r, z> with r = aux, the V-cycle's
// input, into partial[rhs][block].
template <typename R, int TX, int TT, int MODE, bool NT, typename TI = cpx<R>, typename TO = cpx<R>, int NRB = 1,
          bool GRP = false>
__global__ void __launch_bounds__(kThreads) k_normal_fused(const cpx<R>* __restrict__ U, const TI* __restrict__ x,
                                                           TO* __restrict__ y, int lx, int lt, R diag, R c, R c2,
                                                           cpx<R>* __restrict__ xacc,
                                                           const cpx<R>* __restrict__ aux,
                                                           const double* __restrict__ beta = nullptr,
                                                           double* __restrict__ partial = nullptr,
                                                           BetaFold bf = BetaFold{}, int nrhs = 0,
                                                           Grp g = Grp{}) {
  constexpr int HX = TX + 2, HT = TT + 2;
  constexpr int RG = kThreads / TX;          // row groups
  constexpr int PER = TX * TT / kThreads;    // sites per thread
  static_assert(PER >= 1 && TX * TT % kThreads == 0, "tile shape");
  __shared__ cpx<R> sp[HT * HX * 2];           // psi, halo included: [ht][hx][spin]
  __shared__ cpx<R> sf[TT * TX * 2];           // phi on the tile
  __shared__ cpx<R> sr[2 * TX + 2 * TT];       // projected phi on the ring: xm[TT] xp[TT] tm[TX] tp[TX]

  const int V = lx * lt;
  const int ntx = lx / TX;
  const int tile = fused_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % ntx) * TX, t0 = (tile / ntx) * TT;
  static_assert(NRB == 1 || MODE <= 5, "several right-hand sides per workgroup: epilogues 0-5 only");
  const int nr = nrhs > 0 ? nrhs : (int)gridDim.y * NRB;
  static_assert(!GRP || NRB == 1, "grouped launches take one right-hand side per workgroup");
  if constexpr (GRP) {  // grouped: this column's system
    const int col = blockIdx.y;
    U = static_cast<const cpx<R>*>(g.op[col]);
    diag = (R)g.s[col];
    if (g.c) c = (R)g.c[col];
    if (g.c2) c2 = (R)g.c2[col];
  }
  constexpr int NRING = 2 * TX + 2 * TT;
  static_assert(NRING <= kThreads, "one ring site per thread");

  // MODE 6 with a folded beta: the partial sums of <r, z> are requested first, so that
  // waiting for them later does not wait for the loads issued after them
  constexpr int NBF = kBetaFoldMaxBlocks / kThreads;
  double bre[MODE == 6 ? NBF : 1], bim[MODE == 6 ? NBF : 1];
  if constexpr (MODE == 6) {
    if (bf.part) {
#pragma unroll
      for (int u = 0; u < NBF; ++u) {
        const int i = min((int)threadIdx.x + u * kThreads, bf.nb - 1);
        bre[u] = bf.part[2 * ((size_t)blockIdx.y * bf.nb + i)];
        bim[u] = bf.part[2 * ((size_t)blockIdx.y * bf.nb + i) + 1];
      }
    }
  }

  // ---- links, loaded before psi is staged so that both are in flight together
  const int lxi = threadIdx.x % TX, lti = threadIdx.x / TX;
  cpx<R> ku0[PER], ku1[PER], ku0m[PER], ku1m[PER], f0[PER], f1[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int gx = x0 + lxi, gt = t0 + lti + k * RG;
    const int s = gt * lx + gx;
    ku0[k] = U[s];
    ku1[k] = U[V + s];
    ku0m[k] = U[gt * lx + (gx == 0 ? lx - 1 : gx - 1)];
    ku1m[k] = U[V + (gt == 0 ? lt - 1 : gt - 1) * lx + gx];
  }
  // ring site of this thread (threads 0 .. NRING-1): halo coordinates, the hop it skips, its links
  int rhx = 0, rht = 0, rskip = kSkipNone;
  cpx<R> ru0 = mk<R>(0, 0), ru1 = ru0, ru0m = ru0, ru1m = ru0;
  if (threadIdx.x < NRING) {
    const int i = threadIdx.x;
    if (i < TT) { rhx = 0; rht = i + 1; rskip = kSkipXm; }                        // x = x0 - 1
    else if (i < 2 * TT) { rhx = TX + 1; rht = i - TT + 1; rskip = kSkipXp; }     // x = x0 + TX
    else if (i < 2 * TT + TX) { rhx = i - 2 * TT + 1; rht = 0; rskip = kSkipTm; }  // t = t0 - 1
    else { rhx = i - 2 * TT - TX + 1; rht = TT + 1; rskip = kSkipTp; }             // t = t0 + TT
    int gx = x0 + rhx - 1, gt = t0 + rht - 1;
    gx = gx < 0 ? gx + lx : (gx >= lx ? gx - lx : gx);
    gt = gt < 0 ? gt + lt : (gt >= lt ? gt - lt : gt);
    const int s = gt * lx + gx;
    if (rskip != kSkipXp) ru0 = U[s];
    if (rskip != kSkipXm) ru0m = U[gt * lx + (gx == 0 ? lx - 1 : gx - 1)];
    if (rskip != kSkipTp) ru1 = U[V + s];
    if (rskip != kSkipTm) ru1m = U[V + (gt == 0 ? lt - 1 : gt - 1) * lx + gx];
  }

  // NRB right-hand sides per workgroup reuse the links loaded above (their psi
  // staging, D and D^H run once per right-hand side, as with NRB = 1)
#pragma unroll 1
  for (int q = 0; q < NRB; ++q) {
    const int rhs = (int)blockIdx.y * NRB + q;
    if (rhs >= nr) break;  // uniform over the workgroup
    const size_t off = (size_t)rhs * 2 * V;
    const TI* __restrict__ xb = x + off;
    // the epilogue's other operand (xacc for a smoother step, aux for a residual), also early
    cpx<R> ep0[PER], ep1[PER];
    cpx<R> ea0[MODE == 7 ? PER : 1], ea1[MODE == 7 ? PER : 1];  // MODE 7: the V-cycle's input r
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const size_t i0 = off + 2 * (size_t)((t0 + lti + k * RG) * lx + x0 + lxi);
      if (MODE == 1 || MODE == 4 || MODE == 7) { ep0[k] = xacc[i0]; ep1[k] = xacc[i0 + 1]; }
      if (MODE == 2) { ep0[k] = aux[i0]; ep1[k] = aux[i0 + 1]; }
      if (MODE == 7) { ea0[k] = aux[i0]; ea1[k] = aux[i0 + 1]; }
    }
    // ---- stage psi (tile + halo): every load is issued before the first LDS write,
    // so a workgroup waits for one memory latency, not one per pass
    constexpr int NSP = HT * HX * 2, NPASS = (NSP + kThreads - 1) / kThreads;
    TI stage[NPASS];  // raw stored values: widened only after every load has been issued
    cpx<R> stage2[MODE == 6 ? NPASS : 1];
#pragma unroll
    for (int j = 0; j < NPASS; ++j) {
      const int i = threadIdx.x + j * kThreads;
      if (i < NSP) {
        const int comp = i & 1, site = i >> 1;
        const int ht = site / HX, hx = site - ht * HX;
        int gx = x0 + hx - 1, gt = t0 + ht - 1;
        gx = gx < 0 ? gx + lx : (gx >= lx ? gx - lx : gx);
        gt = gt < 0 ? gt + lt : (gt >= lt ? gt - lt : gt);
        stage[j] = xb[2 * (gt * lx + gx) + comp];
        if constexpr (MODE == 6) stage2[j] = aux[off + 2 * (gt * lx + gx) + comp];
      }
    }
    R bt = 0;
    if constexpr (MODE == 6) {
      if (bf.part) {  // beta from the partial sums of <r, z>, in the order of the separate pass
        __shared__ double sb[2 * (kThreads / 64)];
        const int j = blockIdx.y;
        double re = 0, im = 0;
#pragma unroll
        for (int u = 0; u < NBF; ++u) {
          if ((int)threadIdx.x + u * kThreads < bf.nb) {
            re += bre[u];
            im += bim[u];
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          re += __shfl_xor(re, o, 64);
          im += __shfl_xor(im, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
          sb[2 * (threadIdx.x >> 6)] = re;
          sb[2 * (threadIdx.x >> 6) + 1] = im;
        }
        __syncthreads();
        re = 0;
        im = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
          re += sb[2 * w];
          im += sb[2 * w + 1];
        }
        double be = 0;
        if (bf.rz_old && bf.active[j] && bf.rz_old[2 * j] != 0) be = re / bf.rz_old[2 * j];
        bt = (R)be;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          const bool keep = bf.rz_old && !bf.active[j];
          bf.rz_new[2 * j] = keep ? bf.rz_old[2 * j] : re;
          bf.rz_new[2 * j + 1] = keep ? bf.rz_old[2 * j + 1] : im;
        }
      } else {
        bt = (R)beta[blockIdx.y];
      }
    }
#pragma unroll
    for (int j = 0; j < NPASS; ++j) {
      const int i = threadIdx.x + j * kThreads;
      if constexpr (MODE == 6) {
        // p = z + beta p_old; p = z where beta = 0 (p_old is not read into the sum then)
        if (i < NSP) sp[i] = bt != (R)0 ? widen(stage[j]) + bt * stage2[j] : widen(stage[j]);
      } else {
        if (i < NSP) sp[i] = widen(stage[j]);
      }
    }
    __syncthreads();

    auto P = [&](int ht, int hx, int comp) -> cpx<R> { return sp[(ht * HX + hx) * 2 + comp]; };
    const R half = (R)0.5;

    // D (or a projection of it) at halo coordinates (hx, ht), global (gx, gt).
    auto d_at = [&](int hx, int ht, cpx<R> u0, cpx<R> u1, cpx<R> u0m, cpx<R> u1m, int skip, cpx<R>& o0,
                    cpx<R>& o1) {
      cpx<R> s0 = mk<R>(0, 0), s1 = mk<R>(0, 0);
      if (skip != kSkipXp) hop_acc<R, false>(s0, s1, 0, u0, P(ht, hx + 1, 0), P(ht, hx + 1, 1));
      if (skip != kSkipXm) hop_acc<R, false>(s0, s1, 1, cj(u0m), P(ht, hx - 1, 0), P(ht, hx - 1, 1));
      if (skip != kSkipTp) hop_acc<R, false>(s0, s1, 2, u1, P(ht + 1, hx, 0), P(ht + 1, hx, 1));
      if (skip != kSkipTm) hop_acc<R, false>(s0, s1, 3, cj(u1m), P(ht - 1, hx, 0), P(ht - 1, hx, 1));
      o0 = diag * P(ht, hx, 0) - half * s0;
      o1 = diag * P(ht, hx, 1) - half * s1;
    };

    // ---- phase 1: phi on the tile ------------------------------------------------
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int r = lti + k * RG;
      d_at(lxi + 1, r + 1, ku0[k], ku1[k], ku0m[k], ku1m[k], kSkipNone, f0[k], f1[k]);
      sf[(r * TX + lxi) * 2] = f0[k];
      sf[(r * TX + lxi) * 2 + 1] = f1[k];
    }
    // ---- phase 1b: projected phi on the ring -------------------------------------
    if (threadIdx.x < NRING) {
      cpx<R> o0, o1;
      d_at(rhx, rht, ru0, ru1, ru0m, ru1m, rskip, o0, o1);
      // D^H at the neighbouring tile site uses: from x0-1 (its -x hop) (1 - s1) -> o0 - o1;
      // from x0+TX (+x hop) (1 + s1) -> o0 + o1; from t0-1 (1 - s2) -> o0 + i o1;
      // from t0+TT (1 + s2) -> o0 - i o1.
      cpx<R> h;
      if (rskip == kSkipXm) h = o0 - o1;
      else if (rskip == kSkipXp) h = o0 + o1;
      else if (rskip == kSkipTm) h = o0 + imul(o1);
      else h = o0 - imul(o1);
      sr[threadIdx.x] = h;
    }
    __syncthreads();

    // ---- phase 2: D^H phi on the tile ---------------------------------------------
    double dre = 0, dim = 0;  // MODE 6: this thread's share of <p, A p>
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int r = lti + k * RG;
      const int gx = x0 + lxi, gt = t0 + r;
      const int s = gt * lx + gx;
      cpx<R> s0 = mk<R>(0, 0), s1 = mk<R>(0, 0);
      // +x neighbour: (1 + s1) U0_s phi_{s+x}
      {
        cpx<R> h;
        if (lxi + 1 < TX) h = sf[(r * TX + lxi + 1) * 2] + sf[(r * TX + lxi + 1) * 2 + 1];
        else h = sr[TT + r];
        h = ku0[k] * h;
        s0 = s0 + h; s1 = s1 + h;
      }
      // -x neighbour: (1 - s1) conj(U0_{s-x}) phi_{s-x}
      {
        cpx<R> h;
        if (lxi > 0) h = sf[(r * TX + lxi - 1) * 2] - sf[(r * TX + lxi - 1) * 2 + 1];
        else h = sr[r];
        h = cj(ku0m[k]) * h;
        s0 = s0 + h; s1 = s1 - h;
      }
      // +t neighbour: (1 + s2) U1_s phi_{s+t}: h = phi0 - i phi1, spread (1, i)
      {
        cpx<R> h;
        if (r + 1 < TT) h = sf[((r + 1) * TX + lxi) * 2] - imul(sf[((r + 1) * TX + lxi) * 2 + 1]);
        else h = sr[2 * TT + TX + lxi];
        h = ku1[k] * h;
        s0 = s0 + h; s1 = s1 + imul(h);
      }
      // -t neighbour: (1 - s2) conj(U1_{s-t}) phi_{s-t}: h = phi0 + i phi1, spread (1, -i)
      {
        cpx<R> h;
        if (r > 0) h = sf[((r - 1) * TX + lxi) * 2] + imul(sf[((r - 1) * TX + lxi) * 2 + 1]);
        else h = sr[2 * TT + lxi];
        h = cj(ku1m[k]) * h;
        s0 = s0 + h; s1 = s1 - imul(h);
      }
      const cpx<R> o0 = diag * f0[k] - half * s0;
      const cpx<R> o1 = diag * f1[k] - half * s1;
      const size_t i0 = off + 2 * (size_t)s, i1 = i0 + 1;
      if (MODE == 0) {
        if constexpr (NT && std::is_same<TO, cpx<R>>::value) {  // streaming output: keep it out of the caches
          __builtin_nontemporal_store(o0.re, &y[i0].re);
          __builtin_nontemporal_store(o0.im, &y[i0].im);
          __builtin_nontemporal_store(o1.re, &y[i1].re);
          __builtin_nontemporal_store(o1.im, &y[i1].im);
        } else {
          stv(y, i0, o0);
          stv(y, i1, o1);
        }
      } else if (MODE == 1 || MODE == 3) {
        const cpx<R> v0 = P(r + 1, lxi + 1, 0), v1 = P(r + 1, lxi + 1, 1);
        xacc[i0] = MODE == 3 ? c * v0 : ep0[k] + c * v0;
        xacc[i1] = MODE == 3 ? c * v1 : ep1[k] + c * v1;
        stv(y, i0, v0 - c * o0);
        stv(y, i1, v1 - c * o1);
      } else if (MODE == 4 || MODE == 5) {
        const cpx<R> v0 = P(r + 1, lxi + 1, 0), v1 = P(r + 1, lxi + 1, 1);
        const cpx<R> a0 = MODE == 5 ? c * v0 : ep0[k] + c * v0;
        const cpx<R> a1 = MODE == 5 ? c * v1 : ep1[k] + c * v1;
        xacc[i0] = a0 + c2 * (v0 - c * o0);
        xacc[i1] = a1 + c2 * (v1 - c * o1);
      } else if (MODE == 7) {
        const cpx<R> v0 = P(r + 1, lxi + 1, 0), v1 = P(r + 1, lxi + 1, 1);
        const cpx<R> z0 = ep0[k] + c * v0 + c2 * (v0 - c * o0);
        const cpx<R> z1 = ep1[k] + c * v1 + c2 * (v1 - c * o1);
        xacc[i0] = z0;
        xacc[i1] = z1;
        const cpx<R> a0 = ea0[k], a1 = ea1[k];
        dre += (double)a0.re * z0.re + (double)a0.im * z0.im + (double)a1.re * z1.re + (double)a1.im * z1.im;
        dim += (double)a0.re * z0.im - (double)a0.im * z0.re + (double)a1.re * z1.im - (double)a1.im * z1.re;
      } else if (MODE == 6) {
        const cpx<R> v0 = P(r + 1, lxi + 1, 0), v1 = P(r + 1, lxi + 1, 1);
        xacc[i0] = v0;
        xacc[i1] = v1;
        stv(y, i0, o0);
        stv(y, i1, o1);
        dre += (double)v0.re * o0.re + (double)v0.im * o0.im + (double)v1.re * o1.re + (double)v1.im * o1.im;
        dim += (double)v0.re * o0.im - (double)v0.im * o0.re + (double)v1.re * o1.im - (double)v1.im * o1.re;
      } else {
        stv(y, i0, ep0[k] - o0);
        stv(y, i1, ep1[k] - o1);
      }
    }
    if constexpr (MODE == 6 || MODE == 7) {
      __shared__ double sred[2 * (kThreads / 64)];
      for (int o = 32; o > 0; o >>= 1) {
        dre += __shfl_xor(dre, o, 64);
        dim += __shfl_xor(dim, o, 64);
      }
      if ((threadIdx.x & 63) == 0) {
        sred[2 * (threadIdx.x >> 6)] = dre;
        sred[2 * (threadIdx.x >> 6) + 1] = dim;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
          a += sred[2 * w];
          b += sred[2 * w + 1];
        }
        const size_t pi = 2 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x);
        partial[pi] = a;
        partial[pi + 1] = b;
      }
    }
    if (NRB > 1) __syncthreads();  // the next right-hand side overwrites sp, sf and sr
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

// With at least kFusedNRB right-hand sides on a lattice of at least kFusedNRBSites
// sites a workgroup takes kFusedNRB of them in turn and loads its links once (96 ->
// 64 + 32 / kFusedNRB bytes per site and right-hand side in FP64); each column's
// arithmetic is the same either way.  Measured on MI355X: 2048^2, 64 RHS: FP64 4.29
// -> 3.82 ms, FP32 2.24 -> 1.87 ms; at 512^2 (cache-resident, and the loop halves the
// waves per SIMD) FP64 32 RHS ran 0.099 -> 0.112 ms, so small lattices keep one
// right-hand side per workgroup.  Dispatching a tile's right-hand sides next to each
// other instead (links from L2, one per workgroup) was slower at both sizes.
constexpr int kFusedNRB = 4;
constexpr long kFusedNRBSites = 1L << 20;

template <typename R, int TX, int TT, bool NT>
void launch_fused(const cpx<R>* U, const cpx<R>* x, cpx<R>* y, int lx, int lt, double diag, int nrhs, int mode,
                  double c, double c2, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st, const Grp& g) {
  const int tiles = (lx / TX) * (lt / TT);
  with_mode(mode, [&](auto m) {
    constexpr int M = decltype(m)::v;
    if (g.op) {
      hipLaunchKernelGGL((k_normal_fused<R, TX, TT, M, NT, cpx<R>, cpx<R>, 1, true>), dim3(tiles, nrhs),
                         dim3(kThreads), 0, st, U, x, y, lx, lt, (R)diag, (R)c, (R)c2, xacc, aux, nullptr, nullptr,
                         BetaFold{}, 0, g);
    } else if (nrhs >= kFusedNRB && (long)lx * lt >= kFusedNRBSites) {
      dim3 grid(tiles, (nrhs + kFusedNRB - 1) / kFusedNRB);
      hipLaunchKernelGGL((k_normal_fused<R, TX, TT, M, NT, cpx<R>, cpx<R>, kFusedNRB>), grid, dim3(kThreads), 0, st,
                         U, x, y, lx, lt, (R)diag, (R)c, (R)c2, xacc, aux, nullptr, nullptr, BetaFold{}, nrhs);
    } else {
      hipLaunchKernelGGL((k_normal_fused<R, TX, TT, M, NT>), dim3(tiles, nrhs), dim3(kThreads), 0, st, U, x, y, lx,
                         lt, (R)diag, (R)c, (R)c2, xacc, aux);
    }
  });
  HIPCHECK(hipGetLastError());
}

template <typename R, int TX, int TT, bool NT>
void launch_cg_step_t(const cpx<R>* U, const cpx<R>* z, const cpx<R>* p_old, cpx<R>* p, cpx<R>* q, int lx, int lt,
                      double diag, int nrhs, const double* beta, double* partial, hipStream_t st,
                      const BetaFold& bf, const Grp& g) {
  dim3 grid((lx / TX) * (lt / TT), nrhs);
  if (g.op)
    hipLaunchKernelGGL((k_normal_fused<R, TX, TT, 6, NT, cpx<R>, cpx<R>, 1, true>), grid, dim3(kThreads), 0, st, U, z,
                       q, lx, lt, (R)diag, (R)0, (R)0, p, p_old, beta, partial, bf, 0, g);
  else
    hipLaunchKernelGGL((k_normal_fused<R, TX, TT, 6, NT>), grid, dim3(kThreads), 0, st, U, z, q, lx, lt, (R)diag,
                       (R)0, (R)0, p, p_old, beta, partial, bf, 0, g);
  HIPCHECK(hipGetLastError());
}

// Tile shape of the fused kernel, from measurements on MI355X at 256^2 to 4096^2
// (all loads of a workgroup issued before its first wait): 64x8 with non-temporal
// output stores is the fastest in both precisions once the lattice has at least
// 256 (FP64) or 1024 (FP32) such tiles; smaller lattices run faster on 16x16 tiles
// (one site per thread, twice the workgroups).  Shapes that do not divide the
// lattice fall back to the next one that does; kTileNone means no tile fits and A
// is applied as D followed by D^H.
enum { kTileNone = 0, kT64x4, kT64x8nt, kT32x16nt, kT32x8, kT16x16 };

template <typename R>
int fused_shape(int lx, int lt) {
  const bool small = (long)lx * lt / 512 < (sizeof(R) == 8 ? 256 : 1024);
  int pref[4] = {kT64x8nt, kT32x16nt, kT64x4, kT32x8};
  if (small) {
    pref[0] = kT16x16;
    pref[1] = kT32x8;
    pref[2] = kT64x8nt;
    pref[3] = kT32x16nt;
  }
  auto fits = [&](int sh) {
    switch (sh) {
      case kT64x4: return lx % 64 == 0 && lt % 4 == 0;
      case kT64x8nt: return lx % 64 == 0 && lt % 8 == 0;
      case kT32x16nt: return lx % 32 == 0 && lt % 16 == 0;
      case kT32x8: return lx % 32 == 0 && lt % 8 == 0;
      case kT16x16: return lx % 16 == 0 && lt % 16 == 0;
    }
    return false;
  };
  for (int sh : pref)
    if (fits(sh)) return sh;
  return fits(kT16x16) ? kT16x16 : kTileNone;
}

template <typename R>
void launch_normal(const cpx<R>* U, const cpx<R>* x, cpx<R>* y, cpx<R>* tmp, int lx, int lt, double diag,
                   int nrhs, int mode, double c, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st, double c2,
                   const Grp& g) {
  switch (fused_shape<R>(lx, lt)) {
    case kT64x4: launch_fused<R, 64, 4, false>(U, x, y, lx, lt, diag, nrhs, mode, c, c2, xacc, aux, st, g); return;
    case kT64x8nt: launch_fused<R, 64, 8, true>(U, x, y, lx, lt, diag, nrhs, mode, c, c2, xacc, aux, st, g); return;
    case kT32x16nt: launch_fused<R, 32, 16, true>(U, x, y, lx, lt, diag, nrhs, mode, c, c2, xacc, aux, st, g); return;
    case kT32x8: launch_fused<R, 32, 8, false>(U, x, y, lx, lt, diag, nrhs, mode, c, c2, xacc, aux, st, g); return;
    case kT16x16: launch_fused<R, 16, 16, false>(U, x, y, lx, lt, diag, nrhs, mode, c, c2, xacc, aux, st, g); return;
    default: break;
  }
  if (g.op) throw Error(-1, "grouped fine operator needs a fused tile shape");
  launch_wilson<R>(U, x, tmp, lx, lt, diag, nrhs, false, st);
  const int V = lx * lt;
  dim3 grid((V + kThreads - 1) / kThreads, nrhs);
  with_mode(mode, [&](auto m) {
    hipLaunchKernelGGL((k_normal2<R, decltype(m)::v>), grid, dim3(kThreads), 0, st, U, tmp, x, y, lx, lt, (R)diag,
                       (R)c, (R)c2, xacc, aux);
  });
  HIPCHECK(hipGetLastError());
}

template <typename R, int TX, int TT, bool NT>
void launch_vcycle_end_t(const cpx<R>* U, const cpx<R>* v, cpx<R>* z, const cpx<R>* r, int lx, int lt, double diag,
                         int nrhs, double c, double c2, double* partial, hipStream_t st, const Grp& g) {
  dim3 grid((lx / TX) * (lt / TT), nrhs);
  if (g.op)
    hipLaunchKernelGGL((k_normal_fused<R, TX, TT, 7, NT, cpx<R>, cpx<R>, 1, true>), grid, dim3(kThreads), 0, st, U, v,
                       static_cast<cpx<R>*>(nullptr), lx, lt, (R)diag, (R)c, (R)c2, z, r,
                       static_cast<const double*>(nullptr), partial, BetaFold{}, 0, g);
  else
    hipLaunchKernelGGL((k_normal_fused<R, TX, TT, 7, NT>), grid, dim3(kThreads), 0, st, U, v,
                       static_cast<cpx<R>*>(nullptr), lx, lt, (R)diag, (R)c, (R)c2, z, r,
                       static_cast<const double*>(nullptr), partial, BetaFold{}, 0, g);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_vcycle_end(const cpx<R>* U, const cpx<R>* v, cpx<R>* z, const cpx<R>* r, int lx, int lt, double diag,
                       int nrhs, double c, double c2, double* partial, hipStream_t st, const Grp& g) {
  switch (fused_shape<R>(lx, lt)) {
    case kT64x4: launch_vcycle_end_t<R, 64, 4, false>(U, v, z, r, lx, lt, diag, nrhs, c, c2, partial, st, g); return;
    case kT64x8nt: launch_vcycle_end_t<R, 64, 8, true>(U, v, z, r, lx, lt, diag, nrhs, c, c2, partial, st, g); return;
    case kT32x16nt: launch_vcycle_end_t<R, 32, 16, true>(U, v, z, r, lx, lt, diag, nrhs, c, c2, partial, st, g); return;
    case kT32x8: launch_vcycle_end_t<R, 32, 8, false>(U, v, z, r, lx, lt, diag, nrhs, c, c2, partial, st, g); return;
    case kT16x16: launch_vcycle_end_t<R, 16, 16, false>(U, v, z, r, lx, lt, diag, nrhs, c, c2, partial, st, g); return;
    default: throw Error(-1, "V-cycle end kernel needs a fused tile shape");
  }
}
template void launch_vcycle_end<float>(const z32*, const z32*, z32*, const z32*, int, int, double, int, double, double,
                                       double*, hipStream_t, const Grp&);

template <typename R>
int cg_step_blocks(int lx, int lt) {
  switch (fused_shape<R>(lx, lt)) {
    case kT64x4: return (lx / 64) * (lt / 4);
    case kT64x8nt: return (lx / 64) * (lt / 8);
    case kT32x16nt: return (lx / 32) * (lt / 16);
    case kT32x8: return (lx / 32) * (lt / 8);
    case kT16x16: return (lx / 16) * (lt / 16);
    default: return 0;
  }
}

template <typename R>
void launch_cg_step(const cpx<R>* U, const cpx<R>* z, const cpx<R>* p_old, cpx<R>* p, cpx<R>* q, int lx, int lt,
                    double diag, int nrhs, const double* beta, double* partial, hipStream_t st,
                    const BetaFold& bf, const Grp& g) {
  switch (fused_shape<R>(lx, lt)) {
    case kT64x4:
      launch_cg_step_t<R, 64, 4, false>(U, z, p_old, p, q, lx, lt, diag, nrhs, beta, partial, st, bf, g);
      return;
    case kT64x8nt:
      launch_cg_step_t<R, 64, 8, true>(U, z, p_old, p, q, lx, lt, diag, nrhs, beta, partial, st, bf, g);
      return;
    case kT32x16nt:
      launch_cg_step_t<R, 32, 16, true>(U, z, p_old, p, q, lx, lt, diag, nrhs, beta, partial, st, bf, g);
      return;
    case kT32x8:
      launch_cg_step_t<R, 32, 8, false>(U, z, p_old, p, q, lx, lt, diag, nrhs, beta, partial, st, bf, g);
      return;
    case kT16x16:
      launch_cg_step_t<R, 16, 16, false>(U, z, p_old, p, q, lx, lt, diag, nrhs, beta, partial, st, bf, g);
      return;
    default: throw Error(-1, "CG step kernel needs a fused tile shape");
  }
}
template int cg_step_blocks<float>(int, int);
template void launch_cg_step<float>(const z32*, const z32*, const z32*, z32*, z32*, int, int, double, int,
                                    const double*, double*, hipStream_t, const BetaFold&, const Grp&);

template <int TX, int TT, typename TI, typename TO>
void launch_fused_lp(const z32* U, const TI* x, TO* y, int lx, int lt, double diag, int nrhs, int mode, double c,
                     double c2, z32* xacc, const z32* aux, hipStream_t st) {
  dim3 grid((lx / TX) * (lt / TT), nrhs);
  with_mode(mode, [&](auto m) {
    hipLaunchKernelGGL((k_normal_fused<float, TX, TT, decltype(m)::v, false, TI, TO>), grid, dim3(kThreads), 0, st, U,
                       x, y, lx, lt, (float)diag, (float)c, (float)c2, xacc, aux);
  });
  HIPCHECK(hipGetLastError());
}

bool normal_lp_fits(int lx, int lt) { return lx % 32 == 0 && lt % 16 == 0; }

template <typename TI, typename TO>
void launch_normal_lp(const z32* U, const TI* x, TO* y, int lx, int lt, double diag, int nrhs, int mode, double c,
                      z32* xacc, const z32* aux, hipStream_t st, double c2) {
  if (!normal_lp_fits(lx, lt)) throw Error(-1, "reduced-precision smoother storage needs lx % 32 == 0, lt % 16 == 0");
  launch_fused_lp<32, 16>(U, x, y, lx, lt, diag, nrhs, mode, c, c2, xacc, aux, st);
}

#define INST_LP(TI, TO)                                                                                          \
  template void launch_normal_lp<TI, TO>(const z32*, const TI*, TO*, int, int, double, int, int, double, z32*,   \
                                         const z32*, hipStream_t, double);
INST_LP(z32, bfc)
INST_LP(bfc, bfc)
INST_LP(z32, hfc)
INST_LP(hfc, hfc)
#undef INST_LP

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
                                    const z64*, hipStream_t, double, const Grp&);
template void launch_normal<float>(const z32*, const z32*, z32*, z32*, int, int, double, int, int, double, z32*,
                                   const z32*, hipStream_t, double, const Grp&);
template void launch_prepare_links<double>(const z64*, z64*, int, int, int, hipStream_t);
template void launch_prepare_links<float>(const z64*, z32*, int, int, int, hipStream_t);

}  // namespace smg
