// air_solve / air_solve_adjoint: FGMRES(m) with right preconditioning by one
// lAIR V-cycle (Section 3 coarse-grid correction; Section 4: no
// pre-relaxation, post-relaxation on F points then all points, here F,F,C
// Jacobi sweeps) on the scaled facet system, and the transposed cycle for
// the adjoint.  Also reconstruction and slab coupling.
//
// Sparse kernels: G lanes per CSR row (G chosen from the mean row length),
// partial sums combined with cross-lane shuffles; rows are contiguous, so a
// group reads its row's values and column indices with unit stride.  A
// relaxation sweep on the point set X (F or C) writes a second buffer
// (Jacobi: every update reads the previous iterate) and copies the other
// rows.  The FGMRES orthogonalisation is classical Gram-Schmidt applied
// twice, with multi-vector dot products reduced in a fixed order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "prof.h"
#include "system.h"

namespace ah {

enum { SP_MV = 0, SP_RES = 1, SP_SWEEP = 2, SP_ADDMV = 3, SP_SWEEP_P = 4, SP_SWEEP_LIST = 5, SP_SWEEP_ORD = 6,
       SP_RESTRICT = 7, SP_SO_P = 8, SP_SO_E = 9, SP_SO_C = 10 };

// MODE SP_MV:      y = A x
// MODE SP_RES:     y = b - A x
// MODE SP_SWEEP:   y_i = x_i + omega (b_i - (A x)_i) / d_i  for cf_i == X (all rows if cf null), else x_i
// MODE SP_ADDMV:   y = b + A x
// MODE SP_SWEEP_P: the sweep applied to the interpolated iterate x = P e,
//                  read on the fly as x_j = e[pc[j]] (0 where pc[j] < 0);
//                  rows outside X get x_i = e[pc[i]]
// MODE SP_SWEEP_LIST: the sweep on the rows listed in pc[0..n) only; other
//                  rows of y are not written
// MODE SP_SWEEP_ORD: SP_SWEEP_LIST on a copy of the listed rows stored in
//                  list order: item ii's entries at rp[ii] .. rp[ii + 1]
// y2 (sweeps, optional): the updated rows are also written there.
// A values may be null (all ones).
template <class TA, class TX, class TY, int G, int MODE>
__global__ __launch_bounds__(256) void k_csr(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                             const TA* __restrict__ av, const TX* __restrict__ x,
                                             const TY* __restrict__ b, const TY* __restrict__ d,
                                             const int8_t* __restrict__ cf, int X, TY omega, TY* __restrict__ y,
                                             const int32_t* __restrict__ pc, TY* __restrict__ y2) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ii = gid / G;
  const int g = (int)(gid % G);
  if (ii >= n) return;
  constexpr bool LS = MODE == SP_SWEEP_LIST || MODE == SP_SWEEP_ORD;
  const int64_t i = LS ? (int64_t)pc[ii] : ii;
  constexpr bool SW = MODE == SP_SWEEP || MODE == SP_SWEEP_P || LS;
  const bool active = LS || !SW || !cf || cf[i] == X;
  // the listed sweeps load the row's own x, b and d before the gather
  TY xpre = 0, bpre = 0, dpre = 0;
  if (LS) {
    xpre = (TY)x[i];
    bpre = b[i];
    dpre = d[i];
  }
  TY acc = 0;
  if (active) {
    const int64_t kr = MODE == SP_SWEEP_ORD ? ii : i;
    const int64_t k1 = rp[kr + 1];
    int64_t kb = rp[kr] + g;
    if (MODE != SP_SWEEP_P && av) {
      // four independent column / value / x loads in flight per lane
      TY acc1 = 0, acc2 = 0, acc3 = 0;
      for (; kb + 3 * G < k1; kb += 4 * G) {
        const int32_t c0 = ci[kb], c1 = ci[kb + G], c2 = ci[kb + 2 * G], c3 = ci[kb + 3 * G];
        const TY a0 = (TY)av[kb], a1 = (TY)av[kb + G], a2 = (TY)av[kb + 2 * G], a3 = (TY)av[kb + 3 * G];
        acc += a0 * (TY)x[c0];
        acc1 += a1 * (TY)x[c1];
        acc2 += a2 * (TY)x[c2];
        acc3 += a3 * (TY)x[c3];
      }
      if (kb < k1) {
        // the last one to three entries of the lane in one step: the loads
        // are clamped to the row's last entry (no branch between them) and
        // the entries past the row weigh zero
        const int64_t l = k1 - 1;
        const int64_t q1 = kb + G < l ? kb + G : l, q2 = kb + 2 * G < l ? kb + 2 * G : l;
        const int32_t c0 = ci[kb], c1 = ci[q1], c2 = ci[q2];
        TY a0 = (TY)av[kb], a1 = (TY)av[q1], a2 = (TY)av[q2];
        a1 = kb + G < k1 ? a1 : (TY)0;
        a2 = kb + 2 * G < k1 ? a2 : (TY)0;
        acc += a0 * (TY)x[c0];
        acc1 += a1 * (TY)x[c1];
        acc2 += a2 * (TY)x[c2];
        kb = k1;
      }
      acc += (acc1 + acc2) + acc3;
    }
    for (int64_t k = kb; k < k1; k += G) {
      TY a = av ? (TY)av[k] : (TY)1;
      if (MODE == SP_SWEEP_P) {
        const int32_t c = pc[ci[k]];
        acc += c >= 0 ? a * (TY)x[c] : (TY)0;
      } else {
        acc += a * (TY)x[ci[k]];
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (g != 0) return;
  if (MODE == SP_MV) y[i] = acc;
  else if (MODE == SP_RES) y[i] = b[i] - acc;
  else if (MODE == SP_ADDMV) y[i] = b[i] + acc;
  else {
    TY xi;
    if (MODE == SP_SWEEP_P) {
      const int32_t c = pc[i];
      xi = c >= 0 ? (TY)x[c] : (TY)0;
    } else {
      xi = LS ? xpre : (TY)x[i];
    }
    if (active) {
      const TY di = LS ? dpre : d[i];
      const TY bi = LS ? bpre : b[i];
      if (fabs((double)di) >= 1e-30) xi += omega * (bi - acc) / di;
      if (y2) y2[i] = xi;
    }
    y[i] = xi;
  }
}

// Level-0 operator by off-diagonal facet blocks (scaled system: identity
// diagonal blocks).  Scalar row i = R B + m holds, for each of the nb
// off-diagonal blocks of block row R, B contiguous values whose columns are
// B ocol[s] + 0..B-1; one column index serves B values and all B rows of the
// block row, so the row stream is the values alone.  Modes SP_MV, SP_RES and
// SP_SWEEP_LIST as in k_csr, with d_i = 1; SP_SWEEP_ORD: SP_SWEEP_LIST with
// item ii's values at soff[ii] of a copy of the listed rows in list order.
template <class TA, class TX, class TY, int B, int G, int MODE>
__global__ __launch_bounds__(256) void k_fb(int64_t n, const int64_t* __restrict__ optr,
                                            const int32_t* __restrict__ ocol, const TA* __restrict__ ov,
                                            const TX* __restrict__ x, const TY* __restrict__ b, TY omega,
                                            TY* __restrict__ y, const int32_t* __restrict__ list,
                                            TY* __restrict__ y2, const int64_t* __restrict__ soff) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ii = gid / G;
  const int g = (int)(gid % G);
  if (ii >= n) return;
  const int64_t i = MODE == SP_SWEEP_LIST || MODE == SP_SWEEP_ORD ? (int64_t)list[ii] : ii;
  // the row's own x and b, loaded by every lane ahead of the gather
  const TY xi = (TY)x[i];
  const TY bi = MODE == SP_MV ? (TY)0 : b[i];
  const int64_t R = i / B;
  const int m = (int)(i - R * B);
  const int64_t o0 = optr[R];
  const int len = (int)(optr[R + 1] - o0) * B;
  const TA* __restrict__ v = MODE == SP_SWEEP_ORD ? ov + soff[ii] : ov + o0 * (B * B) + (int64_t)m * len;
  const int32_t* __restrict__ cb = ocol + o0;
  TY acc = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  int e = g;
  for (; e + 3 * G < len; e += 4 * G) {
    const int e1 = e + G, e2 = e + 2 * G, e3 = e + 3 * G;
    const int64_t c0 = (int64_t)cb[e / B] * B + e % B, c1 = (int64_t)cb[e1 / B] * B + e1 % B;
    const int64_t c2 = (int64_t)cb[e2 / B] * B + e2 % B, c3 = (int64_t)cb[e3 / B] * B + e3 % B;
    const TY a0 = (TY)v[e], a1 = (TY)v[e1], a2 = (TY)v[e2], a3 = (TY)v[e3];
    acc += a0 * (TY)x[c0];
    acc1 += a1 * (TY)x[c1];
    acc2 += a2 * (TY)x[c2];
    acc3 += a3 * (TY)x[c3];
  }
  for (; e < len; e += G) acc += (TY)v[e] * (TY)x[(int64_t)cb[e / B] * B + e % B];
  acc += (acc1 + acc2) + acc3;
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (g != 0) return;
  acc += xi;
  if (MODE == SP_MV) {
    y[i] = acc;
  } else if (MODE == SP_RES) {
    y[i] = bi - acc;
  } else {
    const TY xn = xi + omega * (bi - acc);
    y[i] = xn;
    if (y2) y2[i] = xn;
  }
}

// A coarse level read by full blocks (every block of block row R, the
// diagonal one included; row m of R at (m nb + s) B + c from the block row's
// value base: voff[R] into the CSR values av where voff[R] >= 0, else ~voff[R]
// into the side array ax): the Jacobi sweep of SP_SWEEP_LIST on the listed
// rows with the diagonal d, as k_csr.  LP lanes per row, a lane per block
// (s = g, g + LP, ...): a lane reads the block's column index, the row's B
// contiguous values of the block and the B contiguous values of x (wide
// loads: a third of the load instructions of a lane per value).  ORD: item
// k's row is described by rec[k] (its values at rec[k].voff of a copy in
// sweep order in av, its blocks from bcol[rec[k].o0]), one load that does
// not wait for the list.  The row's own x, b and d are loaded before the
// gather and a lane takes two blocks per step, so that the loads of a wave
// wait on three latencies rather than one per block; the sum runs in block
// order, as one block at a time would.
template <class TA, class TX, class TY, int B, int LP, bool ORD>
__global__ __launch_bounds__(256) void k_fbr(int64_t n, const int32_t* __restrict__ list,
                                             const int64_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                                             const int64_t* __restrict__ voff, const AhRowRec* __restrict__ rec,
                                             const TA* __restrict__ av, const TA* __restrict__ ax,
                                             const TX* __restrict__ x, const TY* __restrict__ b,
                                             const TY* __restrict__ d, TY omega, TY* __restrict__ y,
                                             TY* __restrict__ y2) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ii = gid / LP;
  const int g = (int)(gid % LP);
  if (ii >= n) return;
  const int64_t i = list[ii];
  int64_t o0;
  int nb;
  const TA* __restrict__ v;
  if (ORD) {
    const AhRowRec r = rec[ii];
    o0 = r.o0;
    nb = r.nb;
    v = av + r.voff;
  } else {
    const int64_t R = i / B;
    const int m = (int)(i - R * B);
    o0 = bptr[R];
    nb = (int)(bptr[R + 1] - o0);
    const int64_t vo = voff[R];
    v = (vo >= 0 ? av + vo : ax + ~vo) + (int64_t)m * nb * B;
  }
  // every lane loads them (one address per row): no branch for the
  // compiler to wait behind
  TY xi = (TY)x[i];
  const TY bi = b[i], di = d[i];
  const int32_t* __restrict__ cb = bcol + o0;
  TY acc = 0;
  int sl = g;
  for (; sl + LP < nb; sl += 2 * LP) {
    const int64_t J0 = cb[sl], J1 = cb[sl + LP];
    const TA* __restrict__ v0 = v + sl * B;
    const TA* __restrict__ v1 = v0 + LP * B;
    TA a0[B], a1[B];
    TX x0[B], x1[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      a0[c] = v0[c];
      a1[c] = v1[c];
    }
#pragma unroll
    for (int c = 0; c < B; ++c) {
      x0[c] = x[J0 * B + c];
      x1[c] = x[J1 * B + c];
    }
#pragma unroll
    for (int c = 0; c < B; ++c) acc += (TY)a0[c] * (TY)x0[c];
#pragma unroll
    for (int c = 0; c < B; ++c) acc += (TY)a1[c] * (TY)x1[c];
  }
  if (sl < nb) {
    const int64_t J = cb[sl];
    const TA* __restrict__ vr = v + sl * B;
#pragma unroll
    for (int c = 0; c < B; ++c) acc += (TY)vr[c] * (TY)x[J * B + c];
  }
#pragma unroll
  for (int o = LP / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LP);
  if (g != 0) return;
  if (fabs((double)di) >= 1e-30) xi += omega * (bi - acc) / di;
  if (y2) y2[i] = xi;
  y[i] = xi;
}

// The same operator by facet block rows: LPB lanes per block row R, a lane
// per off-diagonal block s of the row (s = g, g + LPB, ...).  A lane reads
// the block's column index once, its B values of x once, and the B x B
// values of the block (row m, column c at (m nb + s) B + c), accumulating
// one sum per row of the block row; the B sums are reduced across the
// lanes and lane m mod LPB writes row R B + m.  Each x value is gathered once for
// the B rows that use it (k_fb gathers it once per row).  Items are block
// rows: all of them (SP_MV, SP_RES), or the blocks of a row list made of
// whole blocks in increasing order (SP_SWEEP_LIST: block k is list[k B] / B),
// or (SP_SWEEP_ORD) the block rows list[k] of a copy of the operator stored
// in that order (item k's blocks at optr[k] .. optr[k + 1]); both sweep.
// SP_RESTRICT: the restriction R = [Z I] of block AIR by coarse blocks k,
// Z's blocks at optr[k] .. optr[k + 1], the identity on the fine block
// list[k B] / B: y[k B + m] = x[R B + m] + (Z x)_m.
// SP_SO_P, SP_SO_E, SP_SO_C: SP_SWEEP_ORD where the iterate is P e_c, or
// P e_c on the C blocks and the F blocks' values on the F blocks, with
// e_c = xc and block one-point P (a copy of coarse blocks), read without
// forming P e_c; the F blocks' values are kept compact, F item k's block at
// k B.  SP_SO_P takes column blocks J >= 0 as coarse blocks of xc (J < 0:
// zero) and the own block from xc at own[k]; SP_SO_E and SP_SO_C take
// J >= 0 as compact F block J of x and J < 0 as coarse block ~J of xc, the
// own block from x at k B (SP_SO_E) or, for the C blocks in coarse order,
// from coarse block k of xc (SP_SO_C).  SP_SO_P and SP_SO_E write y compact
// (y2 at the rows' own places), SP_SO_C writes y at the rows' places.  The
// sums are the ones SP_SWEEP_ORD forms on the interpolated vector.
template <class TA, class TX, class TY, int B, int LPB, int MODE>
__global__ __launch_bounds__(256) void k_fbb(int64_t nbr, const int64_t* __restrict__ optr,
                                             const int32_t* __restrict__ ocol, const TA* __restrict__ ov,
                                             const TX* __restrict__ x, const TY* __restrict__ b, TY omega,
                                             TY* __restrict__ y, const int32_t* __restrict__ list,
                                             TY* __restrict__ y2, const TX* __restrict__ xc,
                                             const int32_t* __restrict__ own) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t kk = gid / LPB;
  const int g = (int)(gid % LPB);
  if (kk >= nbr) return;
  constexpr bool SO = MODE == SP_SO_P || MODE == SP_SO_E || MODE == SP_SO_C;
  const int64_t R = MODE == SP_SWEEP_LIST || MODE == SP_RESTRICT ? (int64_t)list[kk * B] / B
                    : MODE == SP_SWEEP_ORD || SO ? (int64_t)list[kk] : kk;
  const int64_t ko = MODE == SP_SWEEP_ORD || MODE == SP_RESTRICT || SO ? kk : R;
  const int64_t o0 = optr[ko];
  const int nb = (int)(optr[ko + 1] - o0);
  const TA* __restrict__ v = ov + o0 * (B * B);
  // the own block's values: from xc (clamped to coarse block 0 and zeroed
  // where P gives none) or from x
  constexpr bool oc = MODE == SP_SO_P || MODE == SP_SO_C;
  const int64_t po = MODE == SP_SO_P ? (int64_t)own[kk] : MODE == SP_SO_C ? kk : 0;
  const TX* __restrict__ xo = oc ? xc + (int64_t)(po >= 0 ? po : 0) * B : x + (MODE == SP_SO_E ? kk : R) * B;
  const bool oz = oc && po < 0;
  // with a lane per row of the block row, its own x and b are loaded before
  // the gather (their latency overlaps it)
  // (fewer lanes than rows, small blocks: every lane loads all B of them)
  constexpr bool PRE = LPB >= B;
  constexpr bool PALL = !PRE && B <= 4;
  constexpr bool NB = MODE != SP_MV && MODE != SP_RESTRICT;
  TY xpre = 0, bpre = 0;
  TY xall[PALL ? B : 1], ball[PALL ? B : 1];
  if (PRE) {
    const int gp = g < B ? g : B - 1;
    const TY t = (TY)xo[gp];   // loaded in every case: no branch before the wait
    xpre = oz ? (TY)0 : t;
    if (NB) bpre = b[R * B + gp];
  }
  if (PALL) {
#pragma unroll
    for (int m = 0; m < B; ++m) {
      const TY t = (TY)xo[m];
      xall[m] = oz ? (TY)0 : t;
      ball[m] = NB ? b[R * B + m] : (TY)0;
    }
  }
  TY acc[B];
#pragma unroll
  for (int m = 0; m < B; ++m) acc[m] = 0;
  for (int sl = g; sl < nb; sl += LPB) {
    const int64_t J = ocol[o0 + sl];
    TY xv[B];
    if (MODE == SP_SO_P) {
      const TX* __restrict__ xs = xc + (J >= 0 ? J : 0) * B;
#pragma unroll
      for (int c = 0; c < B; ++c) {
        const TY t = (TY)xs[c];   // loaded in every case: no branch before the wait
        xv[c] = J >= 0 ? t : (TY)0;
      }
    } else if (MODE == SP_SO_E || MODE == SP_SO_C) {
      const TX* __restrict__ xs = J >= 0 ? x + J * B : xc + (~J) * B;
#pragma unroll
      for (int c = 0; c < B; ++c) xv[c] = (TY)xs[c];
    } else {
#pragma unroll
      for (int c = 0; c < B; ++c) xv[c] = (TY)x[J * B + c];
    }
#pragma unroll
    for (int m = 0; m < B; ++m) {
      const TA* __restrict__ vr = v + ((int64_t)m * nb + sl) * B;
#pragma unroll
      for (int c = 0; c < B; ++c) acc[m] += (TY)vr[c] * xv[c];
    }
  }
#pragma unroll
  for (int m = 0; m < B; ++m)
#pragma unroll
    for (int o = LPB / 2; o > 0; o >>= 1) acc[m] += __shfl_xor(acc[m], o, LPB);
#pragma unroll
  for (int m = 0; m < B; ++m) {
    if (m % LPB != g) continue;      // lane m mod LPB writes row m
    const int64_t i = R * B + m;
    const TY xi = PRE ? xpre : PALL ? xall[PALL ? m : 0] : oz ? (TY)0 : (TY)xo[m];
    const TY bi = PRE ? bpre : PALL ? ball[PALL ? m : 0] : NB ? b[i] : (TY)0;
    const TY a = acc[m] + xi;
    if (MODE == SP_RESTRICT) {
      y[kk * B + m] = a;
    } else if (MODE == SP_MV) {
      y[i] = a;
    } else if (MODE == SP_RES) {
      y[i] = bi - a;
    } else {
      const TY xn = xi + omega * (bi - a);
      y[MODE == SP_SO_P || MODE == SP_SO_E ? kk * B + m : i] = xn;
      if (y2) y2[i] = xn;
    }
  }
}

// One level of the ordered forward sweep on level 0 (flow order of Lemma
// 3.1): x_i <- b_i - sum of a_ij x_j over the off-diagonal blocks (the
// diagonal blocks are the identity), written to xn.  Blocks of earlier
// levels are read from xn (already swept), blocks of the row's own level
// from xo (values before the level: Jacobi inside a level), later levels
// from xn (still equal to xo).  cols holds ~J for a block J on the row's
// level.  rec: one record per item {item, first value slot of its block row,
// blocks in the row, 0}; BLK: items are blocks and row k is
// rec[k / B].x B + k mod B, otherwise items are rows.
template <class TA, class T, int B, int G, bool BLK>
__global__ __launch_bounds__(256) void k_gs_fb(int64_t n, const int4* __restrict__ rec,
                                               const int32_t* __restrict__ cols, const TA* __restrict__ ov,
                                               const T* __restrict__ b, const T* __restrict__ xo, T* xn) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ii = gid / G;
  const int g = (int)(gid % G);
  if (ii >= n) return;
  const int4 r = rec[BLK ? ii / B : ii];
  const int64_t i = BLK ? (int64_t)r.x * B + ii % B : (int64_t)r.x;
  const int m = (int)(i % B);
  const int64_t o0 = r.y;
  const int len = r.z * B;
  const TA* __restrict__ v = ov + o0 * (B * B) + (int64_t)m * len;
  const int32_t* __restrict__ cb = cols + o0;
  T acc = 0, acc1 = 0;
  int e = g;
  for (; e + G < len; e += 2 * G) {
    const int e1 = e + G;
    const int32_t j0 = cb[e / B], j1 = cb[e1 / B];
    const T* s0 = j0 < 0 ? xo : xn;
    const T* s1 = j1 < 0 ? xo : xn;
    acc += (T)v[e] * s0[(int64_t)(j0 < 0 ? ~j0 : j0) * B + e % B];
    acc1 += (T)v[e1] * s1[(int64_t)(j1 < 0 ? ~j1 : j1) * B + e1 % B];
  }
  if (e < len) {
    const int32_t j0 = cb[e / B];
    acc += (T)v[e] * (j0 < 0 ? xo : xn)[(int64_t)(j0 < 0 ? ~j0 : j0) * B + e % B];
  }
  acc += acc1;
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (g == 0) xn[i] = b[i] - acc;
}

// One level k of the transposed (backward) ordered sweep of the adjoint
// cycle, on the rows of A^T (scalar CSR with its diagonal):
// yn_i = yo_i + (g_i - (A^T y~)_i) / d_i, y~ from yo on the row's own level
// (lev of the column's block == k) and from yn elsewhere.
template <class T, int G, bool BLK>
__global__ __launch_bounds__(256) void k_gs_csr(int64_t n, const int32_t* __restrict__ items, int B,
                                                const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                const T* __restrict__ v, const T* __restrict__ d,
                                                const T* __restrict__ g, const int32_t* __restrict__ lev, int k,
                                                const T* __restrict__ yo, T* yn) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ii = gid / G;
  const int lane = (int)(gid % G);
  if (ii >= n) return;
  const int64_t i = BLK ? (int64_t)items[ii / B] * B + ii % B : (int64_t)items[ii];
  T acc = 0;
  for (int64_t q = rp[i] + lane; q < rp[i + 1]; q += G) {
    const int32_t j = ci[q];
    acc += v[q] * (lev[j / B] == k ? yo : yn)[j];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (lane == 0) yn[i] = yo[i] + (g[i] - acc) / d[i];
}

// Coarse end of the cycle in one workgroup: every level from l0 down,
// one row per thread, phases separated by workgroup barriers.
template <class T>
struct TLv;
template <>
struct TLv<double> {
  __device__ static const double* A(const TailLevel& L) { return L.v; }
  __device__ static const double* AT(const TailLevel& L) { return L.ATv; }
  __device__ static const double* R(const TailLevel& L) { return L.Rv; }
  __device__ static const double* RT(const TailLevel& L) { return L.RTv; }
  __device__ static const double* d(const TailLevel& L) { return L.d; }
  __device__ static double* b(const TailLevel& L) { return L.b; }
  __device__ static double* x(const TailLevel& L) { return L.x; }
  __device__ static double* y(const TailLevel& L) { return L.y; }
};
template <>
struct TLv<float> {
  __device__ static const float* A(const TailLevel& L) { return L.v32; }
  __device__ static const float* AT(const TailLevel& L) { return L.ATv32; }
  __device__ static const float* R(const TailLevel& L) { return L.Rv32; }
  __device__ static const float* RT(const TailLevel& L) { return L.RTv32; }
  __device__ static const float* d(const TailLevel& L) { return L.d32; }
  __device__ static float* b(const TailLevel& L) { return L.b32; }
  __device__ static float* x(const TailLevel& L) { return L.x32; }
  __device__ static float* y(const TailLevel& L) { return L.y32; }
};

template <class T>
__device__ inline T row_dot(const int64_t* rp, const int32_t* ci, const T* av, const T* x, int64_t i) {
  T s = 0;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += (av ? av[k] : (T)1) * x[ci[k]];
  return s;
}

// Global -> LDS staging for the tail kernel: n elements, eight independent
// loads in flight per thread (the image is re-staged on every cycle, so the
// copy must not be one dependent load per iteration).
template <class D, class S>
__device__ inline void tail_stage(D* __restrict__ dst, const S* __restrict__ src, int n, int t, int NT) {
  int k = t;
  for (; k + 7 * NT < n; k += 8 * NT) {
    S a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = src[k + q * NT];
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[k + q * NT] = (D)a[q];
  }
  for (; k < n; k += NT) dst[k] = (D)src[k];
}

// Lanes per row for a tail phase over n rows of mean length avg: as many as
// the workgroup allows (power of two, at most 32), not more than the row has.
__device__ inline int tail_lanes(int n, int avg, int NT) {
  int g = 1;
  while (g < 32 && 2 * g * n <= NT && g < avg) g *= 2;
  return g;
}

// Run f(G) with G the compile-time lane count for the runtime value g.
template <class F>
__device__ inline void tail_with_lanes(int g, F&& f) {
  switch (g) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 32>{}); break;
  }
}

// Row i of an LDS CSR matrix times x, split over the G lanes of a group
// (lane g takes entries g, g+G, ...); the sum is returned in every lane.
template <int G, class T, class TS>
__device__ inline TS tail_row(const int32_t* rp, const int32_t* ci, const T* av, const T* x, int i, int g) {
  TS s = 0;
  const int k1 = rp[i + 1];
#pragma unroll 4
  for (int k = rp[i] + g; k < k1; k += G) s += (TS)av[k] * (TS)x[ci[k]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
  return s;
}

// The tail's LDS image written to global memory (layout of
// tail_lds_layout): int32 row offsets, operator values, diagonals, C/F flags,
// one-point columns, R, and the coarsest inverse; the work vectors are left
// unset.
template <class T>
__global__ __launch_bounds__(1024) void k_tail_image(const TailLevel* __restrict__ lv, int l0, int nlev,
                                                     const double* __restrict__ cinv, char* __restrict__ img) {
  __shared__ TailLds lo[TAIL_MAX_LEVELS];
  __shared__ int64_t s_cinv;
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  const int last = nlev - 1;
  if (t == 0) {
    int64_t oc = 0;
    tail_lds_layout<(int)sizeof(T)>(lv, l0, nlev, lo, &oc);
    s_cinv = oc;
  }
  __syncthreads();
#define TI_PTR(type, l, f) reinterpret_cast<type*>(img + lo[(l) - l0].f)
  for (int l = l0; l < last; ++l) {
    const TailLevel& L = lv[l];
    const int n = (int)L.n, nc = (int)L.nc, nnz = (int)L.nnz, nnzR = (int)L.nnzR;
    tail_stage(TI_PTR(int32_t, l, rp), L.rp, n + 1, t, NT);
    tail_stage(TI_PTR(int32_t, l, ci), L.ci, nnz, t, NT);
    tail_stage(TI_PTR(T, l, v), TLv<T>::A(L), nnz, t, NT);
    tail_stage(TI_PTR(T, l, d), TLv<T>::d(L), n, t, NT);
    tail_stage(TI_PTR(int8_t, l, cf), L.cf, n, t, NT);
    tail_stage(TI_PTR(int32_t, l, pc), L.pcol, n, t, NT);
    tail_stage(TI_PTR(int32_t, l, Rp), L.Rp, nc + 1, t, NT);
    tail_stage(TI_PTR(int32_t, l, Rc), L.Rc, nnzR, t, NT);
    tail_stage(TI_PTR(T, l, Rv), TLv<T>::R(L), nnzR, t, NT);
  }
#undef TI_PTR
  const int nL = (int)lv[last].n;
  tail_stage(reinterpret_cast<double*>(img + s_cinv), cinv, nL * nL, t, NT);
}

// Forward coarse end of the cycle from an LDS image: every array of levels
// l0 .. nlev-1 and the coarsest inverse are copied into LDS, then the
// restriction, coarsest solve, interpolation and F, F, C sweeps of all these
// levels run out of LDS with workgroup barriers between the phases; each
// phase gives a row to a group of lanes sized to the level.  The result of
// level l0 is written to out.
template <class T>
__global__ __launch_bounds__(1024) void k_tail_lds(const TailLevel* __restrict__ lv, int l0, int nlev,
                                                   const char* __restrict__ img, const T* __restrict__ b_in,
                                                   T* __restrict__ out, int nsw, T omega) {
  extern __shared__ __align__(16) char sm[];
  __shared__ TailLds lo[TAIL_MAX_LEVELS];
  __shared__ int64_t s_cinv, s_bytes;
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  const int last = nlev - 1;
  if (t == 0) {
    int64_t oc = 0;
    s_bytes = tail_lds_layout<(int)sizeof(T)>(lv, l0, nlev, lo, &oc);
    s_cinv = oc;
  }
  __syncthreads();
#define TL_PTR(type, l, f) reinterpret_cast<type*>(sm + lo[(l) - l0].f)
  // stage the image past level l0's input vector in 16-byte chunks, all of a
  // thread's loads issued before its stores; the input goes into that vector
  {
    const uint4* __restrict__ src = reinterpret_cast<const uint4*>(img);
    uint4* dst = reinterpret_cast<uint4*>(sm);
    const int c1 = (int)(s_bytes >> 4);
    int c = (int)(lo[0].x >> 4) + t;
    for (; c + 7 * NT < c1; c += 8 * NT) {
      uint4 a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = src[c + q * NT];
#pragma unroll
      for (int q = 0; q < 8; ++q) dst[c + q * NT] = a[q];
    }
    for (; c < c1; c += NT) dst[c] = src[c];
    tail_stage(TL_PTR(T, l0, b), b_in, (int)lv[l0].n, t, NT);
  }
  const int nL = (int)lv[last].n;
  const double* ci_s = reinterpret_cast<const double*>(sm + s_cinv);
  __syncthreads();
  // restriction down to the coarsest level
  for (int l = l0; l < last; ++l) {
    const int nc = (int)lv[l].nc;
    const int32_t* Rp = TL_PTR(int32_t, l, Rp);
    const int32_t* Rc = TL_PTR(int32_t, l, Rc);
    const T* Rv = TL_PTR(T, l, Rv);
    const T* b = TL_PTR(T, l, b);
    T* cb = TL_PTR(T, l + 1, b);
    const int gR = tail_lanes(nc, nc ? (int)(lv[l].nnzR / nc) : 1, NT);
    tail_with_lanes(gR, [&](auto GC) {
      constexpr int G = decltype(GC)::value;
      const int g = t % G;
      for (int i = t / G; i < nc; i += NT / G) {
        const T r = tail_row<G, T, T>(Rp, Rc, Rv, b, i, g);
        if (g == 0) cb[i] = r;
      }
    });
    __syncthreads();
  }
  // coarsest: y = C^-1 b (FP64 accumulation)
  {
    const T* b = TL_PTR(T, last, b);
    T* z = TL_PTR(T, last, y);
    tail_with_lanes(tail_lanes(nL, nL, NT), [&](auto GC) {
      constexpr int G = decltype(GC)::value;
      const int g = t % G;
      for (int i = t / G; i < nL; i += NT / G) {
        double s = 0.0;
        for (int j = g; j < nL; j += G) s += ci_s[i * nL + j] * (double)b[j];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (g == 0) z[i] = (T)s;
      }
    });
    __syncthreads();
  }
  // up: x = P e_c, then the sweeps ping-pong x -> y -> x -> y
  for (int l = last - 1; l >= l0; --l) {
    const int n = (int)lv[l].n;
    const int32_t* rp = TL_PTR(int32_t, l, rp);
    const int32_t* ci = TL_PTR(int32_t, l, ci);
    const T* v = TL_PTR(T, l, v);
    const T* d = TL_PTR(T, l, d);
    const int8_t* cf = TL_PTR(int8_t, l, cf);
    const int32_t* pc = TL_PTR(int32_t, l, pc);
    const T* bl = TL_PTR(T, l, b);
    const T* ec = TL_PTR(T, l + 1, y);
    T* cur = TL_PTR(T, l, x);
    for (int i = t; i < n; i += NT) cur[i] = pc[i] >= 0 ? ec[pc[i]] : (T)0;
    __syncthreads();
    const int gA = tail_lanes(n, n ? (int)(lv[l].nnz / n) : 1, NT);
    for (int s = 0; s < nsw; ++s) {
      const int X = (nsw == 1 || s < 2) ? 0 : 1;
      T* dst = (s % 2 == 0) ? TL_PTR(T, l, y) : TL_PTR(T, l, x);
      tail_with_lanes(gA, [&](auto GC) {
        constexpr int G = decltype(GC)::value;
        const int g = t % G;
        for (int i = t / G; i < n; i += NT / G) {
          T xi = cur[i];
          if (cf[i] == X) {
            const T di = d[i];
            const T r = tail_row<G, T, T>(rp, ci, v, cur, i, g);
            if (fabs((double)di) >= 1e-30) xi += omega * (bl[i] - r) / di;
          }
          if (g == 0) dst[i] = xi;
        }
      });
      __syncthreads();
      cur = dst;
    }
  }
  // the level-l0 result is in y (odd number of sweeps) or in y (coarsest only)
  {
    const T* r = (l0 == last) ? TL_PTR(T, last, y) : TL_PTR(T, l0, y);
    for (int i = t; i < (int)lv[l0].n; i += NT) out[i] = r[i];
  }
#undef TL_PTR
}

// The transposed tail's LDS image in global memory (layout of
// tail_lds_layout_t): A^T, the diagonal, C/F flags, P^T and R^T of every
// tail level but the coarsest, then the coarsest inverse.
template <class T>
__global__ __launch_bounds__(1024) void k_tail_image_t(const TailLevel* __restrict__ lv, int l0, int nlev,
                                                       const double* __restrict__ cinv, char* __restrict__ img) {
  __shared__ TailLdsT lo[TAIL_MAX_LEVELS];
  __shared__ int64_t s_cinv;
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  const int last = nlev - 1;
  if (t == 0) {
    int64_t oc = 0;
    tail_lds_layout_t<(int)sizeof(T)>(lv, l0, nlev, lo, &oc);
    s_cinv = oc;
  }
  __syncthreads();
#define TI_PTR(type, l, f) reinterpret_cast<type*>(img + lo[(l) - l0].f)
  for (int l = l0; l < last; ++l) {
    const TailLevel& L = lv[l];
    const int n = (int)L.n, nc = (int)L.nc, nnz = (int)L.nnz, nnzR = (int)L.nnzR, nnzP = (int)L.nnzP;
    tail_stage(TI_PTR(int32_t, l, ATp), L.ATp, n + 1, t, NT);
    tail_stage(TI_PTR(int32_t, l, ATc), L.ATc, nnz, t, NT);
    tail_stage(TI_PTR(T, l, ATv), TLv<T>::AT(L), nnz, t, NT);
    tail_stage(TI_PTR(T, l, d), TLv<T>::d(L), n, t, NT);
    tail_stage(TI_PTR(int8_t, l, cf), L.cf, n, t, NT);
    tail_stage(TI_PTR(int32_t, l, PTp), L.PTp, nc + 1, t, NT);
    tail_stage(TI_PTR(int32_t, l, PTc), L.PTc, nnzP, t, NT);
    tail_stage(TI_PTR(int32_t, l, RTp), L.RTp, n + 1, t, NT);
    tail_stage(TI_PTR(int32_t, l, RTc), L.RTc, nnzR, t, NT);
    tail_stage(TI_PTR(T, l, RTv), TLv<T>::RT(L), nnzR, t, NT);
  }
#undef TI_PTR
  const int nL = (int)lv[last].n;
  tail_stage(reinterpret_cast<double*>(img + s_cinv), cinv, nL * nL, t, NT);
}

// Transposed coarse end of the cycle (adjoint) from an LDS image: on each
// level the first sweep from zero (C points; F points with one sweep), the
// F sweeps with A^T, the residual restricted by P^T; the transposed
// coarsest solve; then on the way up y + R^T e_c.  The result of level l0
// is written to out.
template <class T>
__global__ __launch_bounds__(1024) void k_tail_lds_t(const TailLevel* __restrict__ lv, int l0, int nlev,
                                                     const char* __restrict__ img, const T* __restrict__ g_in,
                                                     T* __restrict__ out, int nsw, T omega) {
  extern __shared__ __align__(16) char sm[];
  __shared__ TailLdsT lo[TAIL_MAX_LEVELS];
  __shared__ int64_t s_cinv, s_bytes;
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  const int last = nlev - 1;
  if (t == 0) {
    int64_t oc = 0;
    s_bytes = tail_lds_layout_t<(int)sizeof(T)>(lv, l0, nlev, lo, &oc);
    s_cinv = oc;
  }
  __syncthreads();
#define TL_PTR(type, l, f) reinterpret_cast<type*>(sm + lo[(l) - l0].f)
  {
    const uint4* __restrict__ src = reinterpret_cast<const uint4*>(img);
    uint4* dst = reinterpret_cast<uint4*>(sm);
    const int c1 = (int)(s_bytes >> 4);
    int c = (int)(lo[0].x >> 4) + t;
    for (; c + 7 * NT < c1; c += 8 * NT) {
      uint4 a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = src[c + q * NT];
#pragma unroll
      for (int q = 0; q < 8; ++q) dst[c + q * NT] = a[q];
    }
    for (; c < c1; c += NT) dst[c] = src[c];
    tail_stage(TL_PTR(T, l0, g), g_in, (int)lv[l0].n, t, NT);
  }
  const int nL = (int)lv[last].n;
  const double* ci_s = reinterpret_cast<const double*>(sm + s_cinv);
  __syncthreads();
  for (int l = l0; l < last; ++l) {
    const int n = (int)lv[l].n, nc = (int)lv[l].nc;
    const int32_t* rp = TL_PTR(int32_t, l, ATp);
    const int32_t* ci = TL_PTR(int32_t, l, ATc);
    const T* v = TL_PTR(T, l, ATv);
    const T* d = TL_PTR(T, l, d);
    const int8_t* cf = TL_PTR(int8_t, l, cf);
    const T* g = TL_PTR(T, l, g);
    T* x = TL_PTR(T, l, x);
    T* y = TL_PTR(T, l, y);
    const int X0 = nsw == 1 ? 0 : 1;
    for (int i = t; i < n; i += NT) {
      const T di = d[i];
      x[i] = (cf[i] == X0 && fabs((double)di) >= 1e-30) ? omega * g[i] / di : (T)0;
    }
    __syncthreads();
    const int gA = tail_lanes(n, n ? (int)(lv[l].nnz / n) : 1, NT);
    // F sweeps x -> y -> x
    for (int s = 1; s < nsw; ++s) {
      const T* cur = (s == 1) ? x : y;
      T* dst = (s == 1) ? y : x;
      tail_with_lanes(gA, [&](auto GC) {
        constexpr int G = decltype(GC)::value;
        const int gl = t % G;
        for (int i = t / G; i < n; i += NT / G) {
          T yi = cur[i];
          if (cf[i] == 0) {
            const T di = d[i];
            const T r = tail_row<G, T, T>(rp, ci, v, cur, i, gl);
            if (fabs((double)di) >= 1e-30) yi += omega * (g[i] - r) / di;
          }
          if (gl == 0) dst[i] = yi;
        }
      });
      __syncthreads();
    }
    // residual into y, restricted by P^T into the next level's g
    tail_with_lanes(gA, [&](auto GC) {
      constexpr int G = decltype(GC)::value;
      const int gl = t % G;
      for (int i = t / G; i < n; i += NT / G) {
        const T r = tail_row<G, T, T>(rp, ci, v, x, i, gl);
        if (gl == 0) y[i] = g[i] - r;
      }
    });
    __syncthreads();
    const int32_t* pp = TL_PTR(int32_t, l, PTp);
    const int32_t* pc = TL_PTR(int32_t, l, PTc);
    T* cg = TL_PTR(T, l + 1, g);
    const int gP = tail_lanes(nc, nc ? (int)(lv[l].nnzP / nc) : 1, NT);
    tail_with_lanes(gP, [&](auto GC) {
      constexpr int G = decltype(GC)::value;
      const int gl = t % G;
      for (int c = t / G; c < nc; c += NT / G) {
        T s = 0;
        for (int k = pp[c] + gl; k < pp[c + 1]; k += G) s += y[pc[k]];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (gl == 0) cg[c] = s;
      }
    });
    __syncthreads();
  }
  // coarsest: e = C^-T g (FP64 accumulation), into the coarsest x (or out)
  {
    const T* g = TL_PTR(T, last, g);
    T* e = TL_PTR(T, last, x);
    tail_with_lanes(tail_lanes(nL, nL, NT), [&](auto GC) {
      constexpr int G = decltype(GC)::value;
      const int gl = t % G;
      for (int i = t / G; i < nL; i += NT / G) {
        double s = 0.0;
        for (int j = gl; j < nL; j += G) s += ci_s[j * nL + i] * (double)g[j];
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (gl == 0) {
          if (l0 == last) out[i] = (T)s;
          else e[i] = (T)s;
        }
      }
    });
    __syncthreads();
  }
  // up: out_l = y_l + R^T e_c (y_l is in x), into the level's g (out at l0)
  for (int l = last - 1; l >= l0; --l) {
    const int n = (int)lv[l].n;
    const T* ec = (l + 1 == last) ? TL_PTR(T, last, x) : TL_PTR(T, l + 1, g);
    const int32_t* rp = TL_PTR(int32_t, l, RTp);
    const int32_t* ci = TL_PTR(int32_t, l, RTc);
    const T* v = TL_PTR(T, l, RTv);
    const T* yl = TL_PTR(T, l, x);
    T* gl_out = TL_PTR(T, l, g);
    const int gR = tail_lanes(n, n ? (int)(lv[l].nnzR / n) : 1, NT);
    tail_with_lanes(gR, [&](auto GC) {
      constexpr int G = decltype(GC)::value;
      const int gl = t % G;
      for (int i = t / G; i < n; i += NT / G) {
        const T r = tail_row<G, T, T>(rp, ci, v, ec, i, gl);
        if (gl == 0) {
          if (l == l0) out[i] = yl[i] + r;
          else gl_out[i] = yl[i] + r;
        }
      }
    });
    __syncthreads();
  }
#undef TL_PTR
}

template <class T, bool TR>
__global__ __launch_bounds__(1024) void k_tail(const TailLevel* __restrict__ lv, int l0, int nlev,
                                               const double* __restrict__ cinv, const T* b_in, T* out, int nsw,
                                               T omega) {
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  const int last = nlev - 1;
  if (!TR) {
    const T* b = b_in;
    for (int l = l0; l < last; ++l) {
      const TailLevel& L = lv[l];
      T* cb = TLv<T>::b(lv[l + 1]);
      for (int64_t i = t; i < L.nc; i += NT) cb[i] = row_dot<T>(L.Rp, L.Rc, TLv<T>::R(L), b, i);
      __syncthreads();
      b = cb;
    }
    {
      const TailLevel& LL = lv[last];
      T* z = last == l0 ? out : TLv<T>::y(LL);
      for (int64_t i = t; i < LL.n; i += NT) {
        double s = 0.0;
        for (int64_t j = 0; j < LL.n; ++j) s += cinv[i * LL.n + j] * (double)b[j];
        z[i] = (T)s;
      }
      __syncthreads();
    }
    for (int l = last - 1; l >= l0; --l) {
      const TailLevel& L = lv[l];
      const T* bl = l == l0 ? b_in : TLv<T>::b(L);
      T* outl = l == l0 ? out : TLv<T>::y(L);
      const T* ec = TLv<T>::y(lv[l + 1]);
      T* cur = TLv<T>::x(L);
      T* alt = TLv<T>::y(L);
      for (int64_t i = t; i < L.n; i += NT) cur[i] = L.pcol[i] >= 0 ? ec[L.pcol[i]] : (T)0;
      __syncthreads();
      for (int s = 0; s < nsw; ++s) {
        const int X = (nsw == 1 || s < 2) ? 0 : 1;
        T* dst = s == nsw - 1 ? outl : alt;
        for (int64_t i = t; i < L.n; i += NT) {
          T xi = cur[i];
          if (L.cf[i] == X) {
            T di = TLv<T>::d(L)[i];
            if (fabs((double)di) >= 1e-30) xi += omega * (bl[i] - row_dot<T>(L.rp, L.ci, TLv<T>::A(L), cur, i)) / di;
          }
          dst[i] = xi;
        }
        __syncthreads();
        alt = cur;
        cur = dst;
      }
    }
  } else {
    const T* g = b_in;
    for (int l = l0; l < last; ++l) {
      const TailLevel& L = lv[l];
      T* cur = TLv<T>::x(L);
      T* alt = TLv<T>::y(L);
      for (int64_t i = t; i < L.n; i += NT) cur[i] = 0;
      __syncthreads();
      for (int s = 3 - nsw; s < 3; ++s) {
        const int X = s == 0 ? 1 : 0;   // C, F, F
        for (int64_t i = t; i < L.n; i += NT) {
          T yi = cur[i];
          if (L.cf[i] == X) {
            T di = TLv<T>::d(L)[i];
            if (fabs((double)di) >= 1e-30) yi += omega * (g[i] - row_dot<T>(L.ATp, L.ATc, TLv<T>::AT(L), cur, i)) / di;
          }
          alt[i] = yi;
        }
        __syncthreads();
        T* tmp = cur; cur = alt; alt = tmp;
      }
      for (int64_t i = t; i < L.n; i += NT) alt[i] = g[i] - row_dot<T>(L.ATp, L.ATc, TLv<T>::AT(L), cur, i);
      __syncthreads();
      T* cb = TLv<T>::b(lv[l + 1]);
      for (int64_t c = t; c < L.nc; c += NT) cb[c] = row_dot<T>(L.PTp, L.PTc, (const T*)nullptr, alt, c);
      __syncthreads();
      g = cb;
    }
    {
      const TailLevel& LL = lv[last];
      T* e = last == l0 ? out : TLv<T>::x(LL);
      for (int64_t i = t; i < LL.n; i += NT) {
        double s = 0.0;
        for (int64_t j = 0; j < LL.n; ++j) s += cinv[j * LL.n + i] * (double)g[j];
        e[i] = (T)s;
      }
      __syncthreads();
    }
    for (int l = last - 1; l >= l0; --l) {
      const TailLevel& L = lv[l];
      const T* ec = (l + 1 == last) ? TLv<T>::x(lv[l + 1]) : TLv<T>::b(lv[l + 1]);
      const T* yl = TLv<T>::y(L);   // sweeps start in x and end in y for 1 or 3 sweeps
      T* outl = l == l0 ? out : TLv<T>::b(L);
      for (int64_t i = t; i < L.n; i += NT) outl[i] = yl[i] + row_dot<T>(L.RTp, L.RTc, TLv<T>::RT(L), ec, i);
      __syncthreads();
    }
  }
}

template <class T>
__global__ void k_interp(int64_t n, const int32_t* __restrict__ pcol, const T* __restrict__ ec, T* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = pcol[i];
  x[i] = c >= 0 ? ec[c] : (T)0;
}

// x = y = P e_c (one-point interpolation, both sweep buffers)
template <class T>
__global__ void k_interp2(int64_t n, const int32_t* __restrict__ pcol, const T* __restrict__ ec,
                          T* __restrict__ x, T* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = pcol[i];
  T v = c >= 0 ? ec[c] : (T)0;
  x[i] = v;
  y[i] = v;
}

// First Jacobi sweep of the transposed cycle from y = 0 on the points of
// set X (cf == X): y_X = omega g_X / d_X, zero elsewhere, into both buffers.
template <class T>
__global__ void k_sweep_from_zero(int64_t n, const int8_t* __restrict__ cf, int X, const T* __restrict__ g,
                                  const T* __restrict__ d, T omega, T* __restrict__ x, T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T v = cf[i] == X && fabs((double)d[i]) >= 1e-30 ? omega * g[i] / d[i] : (T)0;
  x[i] = v;
  y[i] = v;
}

static inline int64_t nF0(const AhLevel& L) { return L.n - L.nc; }

// z = C^-1 r (trans = 0) or C^-T r, FP64 coarsest solve; one wave per row.
template <class T>
__global__ __launch_bounds__(64) void k_coarse(int n, const double* __restrict__ Ci, const T* __restrict__ r,
                                               T* __restrict__ z, int trans) {
  const int row = blockIdx.x;
  const int lane = threadIdx.x;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) {
    double c = trans ? Ci[(int64_t)j * n + row] : Ci[(int64_t)row * n + j];
    acc += c * (double)r[j];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) z[row] = (T)acc;
}

template <class TA, class TB>
__global__ void k_cast(int64_t n, const TA* __restrict__ a, TB* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (TB)a[i];
}

// partial[v][blk] = sum over the block's rows of V_v . w (v < k), and
// partial[k][blk] = w . w.  Vectors are rows of V with stride ldv.
constexpr int DOT_T = 256;
constexpr int DOT_V = 4;

__global__ __launch_bounds__(DOT_T) void k_multidot(int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                                                    const double* __restrict__ w, double* __restrict__ partial,
                                                    int nblk) {
  __shared__ double red[DOT_V][DOT_T / 64];
  const int v0 = blockIdx.y * DOT_V;
  double acc[DOT_V] = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * DOT_T + threadIdx.x; i < n; i += (int64_t)nblk * DOT_T) {
    double wi = w[i];
#pragma unroll
    for (int q = 0; q < DOT_V; ++q) {
      int v = v0 + q;
      if (v < k) acc[q] += V[(int64_t)v * ldv + i] * wi;
      else if (v == k) acc[q] += wi * wi;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < DOT_V; ++q) {
    double a = acc[q];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (lane == 0) red[q][wv] = a;
  }
  __syncthreads();
  if (threadIdx.x < DOT_V) {
    int v = v0 + threadIdx.x;
    if (v <= k) {
      double s = 0.0;
      for (int q = 0; q < DOT_T / 64; ++q) s += red[threadIdx.x][q];
      partial[(int64_t)v * nblk + blockIdx.x] = s;
    }
  }
}

__global__ __launch_bounds__(256) void k_reduce_partial(int nblk, const double* __restrict__ partial,
                                                        double* __restrict__ out, int accumulate) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(int64_t)v * nblk + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = accumulate ? out[v] + red[0] : red[0];
}

// hs[v] = sum over b of partial[v][b] for v < nv, into LDS: wave v % 4
// sums a lane-strided slice and reduces it across the wave.  The order is
// fixed, so every block of a launch obtains the same values.
__device__ inline void partials_to_lds(const double* __restrict__ partial, int nblk, int nv, double* hs) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int v = wv; v < nv; v += nw) {
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += partial[(int64_t)v * nblk + b];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) hs[v] = s;
  }
  __syncthreads();
}

// Classical Gram-Schmidt step from the block partials of k_multidot
// (V_v.w for v < k, w.w at k): h = their sums, w -= sum_{v<k} V_v h_v; block
// 0 also stores h[0..k] in hout.  Dynamic LDS: (k+1) doubles.
__global__ __launch_bounds__(DOT_T) void k_maxpy_p(int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ partial, int nblk,
                                                   double* __restrict__ w, double* __restrict__ hout) {
  extern __shared__ double hs[];
  partials_to_lds(partial, nblk, k + 1, hs);
  if (blockIdx.x == 0)
    for (int v = threadIdx.x; v <= k; v += DOT_T) hout[v] = hs[v];
  for (int64_t i = (int64_t)blockIdx.x * DOT_T + threadIdx.x; i < n; i += (int64_t)gridDim.x * DOT_T) {
    double s = 0.0;
    for (int v = 0; v < k; ++v) s += V[(int64_t)v * ldv + i] * hs[v];
    w[i] -= s;
  }
}

// The same step with the block partial sums of the updated w.w written to
// pout[blockIdx.x] (nblk blocks; pout must not overlap partial).
__global__ __launch_bounds__(DOT_T) void k_maxpy_norm(int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ partial, int nblk,
                                                      double* __restrict__ w, double* __restrict__ hout,
                                                      double* __restrict__ pout) {
  extern __shared__ double hs[];
  __shared__ double red[DOT_T / 64];
  partials_to_lds(partial, nblk, k + 1, hs);
  if (blockIdx.x == 0)
    for (int v = threadIdx.x; v <= k; v += DOT_T) hout[v] = hs[v];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * DOT_T + threadIdx.x; i < n; i += (int64_t)nblk * DOT_T) {
    double s = 0.0;
    for (int v = 0; v < k; ++v) s += V[(int64_t)v * ldv + i] * hs[v];
    double wi = w[i] - s;
    w[i] = wi;
    acc += wi * wi;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < DOT_T / 64; ++q) s += red[q];
    pout[blockIdx.x] = s;
  }
}

// Delayed CGS2 (the second projection of each basis vector is done one
// step late, together with the first projection of the next one), dot pass.
// With the j finished basis vectors Q_l = V[l] (l < j), the candidate
// u = V[j] and the new vector w (or none): block partials of Q_l.u at row l,
// Q_l.w at row j + l, then u.u, u.w, w.w at rows 2j, 2j+1, 2j+2.  Blocks
// along y take DD_V basis vectors each; the blocks of y = 0 also form the
// three scalars.
constexpr int DD_V = 8;

__global__ __launch_bounds__(256) void k_dcgs_dot(int64_t n, int j, const double* __restrict__ V,
                                                  const double* __restrict__ w, double* __restrict__ partial,
                                                  int nblk) {
  __shared__ double red[2 * DD_V + 3][4];
  const int l0 = blockIdx.y * DD_V;
  const int nl = min(DD_V, j - l0);
  const double* __restrict__ u = V + (int64_t)j * n;
  const bool first = blockIdx.y == 0;
  double aa[DD_V], cc[DD_V];
#pragma unroll
  for (int q = 0; q < DD_V; ++q) aa[q] = cc[q] = 0.0;
  double su = 0.0, sw = 0.0, ww = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)nblk * 256) {
    const double ui = u[i];
    const double wi = w ? w[i] : 0.0;
#pragma unroll
    for (int q = 0; q < DD_V; ++q)
      if (q < nl) {
        const double qv = V[(int64_t)(l0 + q) * n + i];
        aa[q] += qv * ui;
        cc[q] += qv * wi;
      }
    if (first) {
      su += ui * ui;
      sw += ui * wi;
      ww += wi * wi;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  auto wave_sum = [&](double a) {
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
  };
#pragma unroll
  for (int q = 0; q < DD_V; ++q) {
    const double a = wave_sum(aa[q]);
    const double c = wave_sum(cc[q]);
    if (lane == 0) { red[q][wv] = a; red[DD_V + q][wv] = c; }
  }
  {
    const double a = wave_sum(su), b = wave_sum(sw), c = wave_sum(ww);
    if (lane == 0) { red[2 * DD_V][wv] = a; red[2 * DD_V + 1][wv] = b; red[2 * DD_V + 2][wv] = c; }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * DD_V + 3) {
    const double s = red[t][0] + red[t][1] + red[t][2] + red[t][3];
    int row = -1;
    if (t < DD_V) { if (t < nl) row = l0 + t; }
    else if (t < 2 * DD_V) { if (t - DD_V < nl) row = j + l0 + (t - DD_V); }
    else if (first) row = 2 * j + (t - 2 * DD_V);
    if (row >= 0) partial[(int64_t)row * nblk + blockIdx.x] = s;
  }
}

// Delayed CGS2, update pass: with coef = [a (j), c (j), d, 1/r], the
// finished vector q = (u - Q a) / r is written over u = V[j] and the next
// candidate (w - Q c - q d) / r into V[j+1] (one read of Q for both).
// Dynamic LDS: 2j + 2 doubles.
__global__ __launch_bounds__(256) void k_dcgs_update(int64_t n, int j, double* __restrict__ V,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ coef) {
  extern __shared__ double cf[];
  for (int t = threadIdx.x; t < 2 * j + 2; t += blockDim.x) cf[t] = coef[t];
  __syncthreads();
  const double d = cf[2 * j], rinv = cf[2 * j + 1];
  double* __restrict__ u = V + (int64_t)j * n;
  double* __restrict__ un = V + (int64_t)(j + 1) * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double sa = 0.0, sc = 0.0;
    for (int l = 0; l < j; ++l) {
      const double qv = V[(int64_t)l * n + i];
      sa += qv * cf[l];
      sc += qv * cf[j + l];
    }
    const double q = (u[i] - sa) * rinv;
    u[i] = q;
    un[i] = (w[i] - sc - q * d) * rinv;
  }
}

// w -= sum_v V_v h_v
template <class TV>
__global__ void k_maxpy(int64_t n, int k, const TV* __restrict__ V, int64_t ldv, const double* __restrict__ h,
                        double* __restrict__ w, double sign) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < k; ++v) s += (double)V[(int64_t)v * ldv + i] * h[v];
  w[i] += sign * s;
}

__global__ void k_scale(int64_t n, const double* __restrict__ a, double s, double* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i] * s;
}

// Block scaling of a right-hand side by D_b^-1 (trans = 0) or D_b^-T.
__global__ void k_blockscale(int64_t nfree, int b, const double* __restrict__ dinv, const double* __restrict__ x,
                             double* __restrict__ y, int trans) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfree * b) return;
  int64_t R = i / b;
  int m = (int)(i % b);
  double s = 0.0;
  for (int k = 0; k < b; ++k)
    s += (trans ? dinv[R * b * b + k * b + m] : dinv[R * b * b + m * b + k]) * x[R * b + k];
  y[i] = s;
}

static inline dim3 g1(int64_t n, int t = 256) { return dim3((unsigned)cdiv(std::max<int64_t>(n, 1), t)); }

static int pick_g(int64_t nnz, int64_t n) {
  double avg = n ? (double)nnz / (double)n : 0.0;
  if (avg < 24) return 4;
  if (avg < 48) return 8;
  if (avg < 80) return 16;
  return 32;
}

template <class TA, class TX, class TY, int MODE>
static ah_status csr_g(int G, int64_t n, const int64_t* rp, const int32_t* ci, const TA* av, const TX* x, const TY* b,
                       const TY* d, const int8_t* cf, int X, TY omega, TY* y, hipStream_t st,
                       const char* tag = nullptr, double bytes = 0.0, const int32_t* pc = nullptr,
                       TY* y2 = nullptr) {
  if (n == 0) return AH_OK;
  ProfScope ps;
  prof_begin(ps, tag, st, bytes);
  dim3 grid((unsigned)cdiv(n * G, 256));
  switch (G) {
    case 2: hipLaunchKernelGGL((k_csr<TA, TX, TY, 2, MODE>), grid, dim3(256), 0, st, n, rp, ci, av, x, b, d, cf, X, omega, y, pc, y2); break;
    case 4: hipLaunchKernelGGL((k_csr<TA, TX, TY, 4, MODE>), grid, dim3(256), 0, st, n, rp, ci, av, x, b, d, cf, X, omega, y, pc, y2); break;
    case 8: hipLaunchKernelGGL((k_csr<TA, TX, TY, 8, MODE>), grid, dim3(256), 0, st, n, rp, ci, av, x, b, d, cf, X, omega, y, pc, y2); break;
    case 16: hipLaunchKernelGGL((k_csr<TA, TX, TY, 16, MODE>), grid, dim3(256), 0, st, n, rp, ci, av, x, b, d, cf, X, omega, y, pc, y2); break;
    default: hipLaunchKernelGGL((k_csr<TA, TX, TY, 32, MODE>), grid, dim3(256), 0, st, n, rp, ci, av, x, b, d, cf, X, omega, y, pc, y2); break;
  }
  prof_end(ps);
  AH_LAUNCHED();
  return AH_OK;
}

// Lanes per row of the facet-block kernels: about eight values per lane
// (the row is one chain of dependent loads per lane, so short rows per lane
// and more rows per wave keep more loads in flight).
static int fb_lanes(int64_t nvals, int64_t n) {
  const double avg = n ? (double)nvals / (double)n : 0.0;
  if (avg < 12) return 2;
  if (avg < 48) return 4;
  if (avg < 96) return 8;
  return 16;
}

template <class TA, class TX, class TY, int MODE, int B>
static void fb_launch(int G, dim3 grid, hipStream_t st, int64_t n, const int64_t* optr, const int32_t* ocol,
                      const TA* ov, const TX* x, const TY* b, TY omega, TY* y, const int32_t* list, TY* y2,
                      const int64_t* soff) {
  switch (G) {
    case 2: hipLaunchKernelGGL((k_fb<TA, TX, TY, B, 2, MODE>), grid, dim3(256), 0, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    case 4: hipLaunchKernelGGL((k_fb<TA, TX, TY, B, 4, MODE>), grid, dim3(256), 0, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    case 8: hipLaunchKernelGGL((k_fb<TA, TX, TY, B, 8, MODE>), grid, dim3(256), 0, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    default: hipLaunchKernelGGL((k_fb<TA, TX, TY, B, 16, MODE>), grid, dim3(256), 0, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
  }
}

// Level-0 rows in the off-diagonal facet-block layout (k_fb): n rows (the
// listed ones for SP_SWEEP_LIST), block size B, G in {2, 4, 8, 16}.
template <class TA, class TX, class TY, int MODE>
static ah_status fb_g(int B, int G, int64_t n, const int64_t* optr, const int32_t* ocol, const TA* ov, const TX* x,
                      const TY* b, TY omega, TY* y, hipStream_t st, const char* tag = nullptr, double bytes = 0.0,
                      const int32_t* list = nullptr, TY* y2 = nullptr, const int64_t* soff = nullptr) {
  if (n == 0) return AH_OK;
  if (G != 2 && G != 4 && G != 8) G = 16;
  ProfScope ps;
  prof_begin(ps, tag, st, bytes);
  const dim3 grid((unsigned)cdiv(n * G, 256));
  switch (B) {
    case 2: fb_launch<TA, TX, TY, MODE, 2>(G, grid, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    case 3: fb_launch<TA, TX, TY, MODE, 3>(G, grid, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    case 4: fb_launch<TA, TX, TY, MODE, 4>(G, grid, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    case 6: fb_launch<TA, TX, TY, MODE, 6>(G, grid, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    case 10: fb_launch<TA, TX, TY, MODE, 10>(G, grid, st, n, optr, ocol, ov, x, b, omega, y, list, y2, soff); break;
    default: set_error("unsupported facet block size %d", B); return AH_EUNSUPPORTED;
  }
  prof_end(ps);
  AH_LAUNCHED();
  return AH_OK;
}

// Sweep of the listed rows of a level read by full blocks (k_fbr); av the
// level's CSR values, ax its side array, in the cycle's precision.  Lanes
// per row: 4 in FP64, 2 in FP32 (C3 level 1, about six blocks per row:
// F sweep 656 / 436 us against 859 / 716 us with 8 lanes; AH_L1LP = 2, 4
// or 8 at setup overrides).
template <class T>
static ah_status fbr_g(const AhLevel& L, const T* av, const T* ax, int64_t n, const int32_t* list, const T* x,
                       const T* b, const T* d, T omega, T* y, hipStream_t st, const char* tag, double bytes,
                       T* y2 = nullptr, const AhRowRec* rec = nullptr) {
  if (n == 0) return AH_OK;
  const int LP = L.blp ? L.blp : sizeof(T) == 8 ? 4 : 2;
  ProfScope ps;
  prof_begin(ps, tag, st, bytes);
  const dim3 grid((unsigned)cdiv(n * LP, 256));
#define FBR(BB, LL)                                                                                         \
  do {                                                                                                      \
    if (rec)                                                                                                \
      hipLaunchKernelGGL((k_fbr<T, T, T, BB, LL, true>), grid, dim3(256), 0, st, n, list, L.bptr, L.bcol,   \
                         (const int64_t*)nullptr, rec, av, ax, x, b, d, omega, y, y2);                      \
    else                                                                                                    \
      hipLaunchKernelGGL((k_fbr<T, T, T, BB, LL, false>), grid, dim3(256), 0, st, n, list, L.bptr, L.bcol,  \
                         L.bvoff, (const AhRowRec*)nullptr, av, ax, x, b, d, omega, y, y2);                 \
  } while (0)
#define FBR_L(BB) switch (LP) { case 2: FBR(BB, 2); break; case 4: FBR(BB, 4); break; default: FBR(BB, 8); break; }
  switch (L.bb) {
    case 2: FBR_L(2); break;
    case 3: FBR_L(3); break;
    case 6: FBR_L(6); break;
    default: prof_end(ps); set_error("unsupported block size %d", L.bb); return AH_EUNSUPPORTED;
  }
#undef FBR_L
#undef FBR
  prof_end(ps);
  AH_LAUNCHED();
  return AH_OK;
}

// Lanes per block row of k_fbb from the mean number of off-diagonal blocks
// per block row (C3: 6 -> 8 lanes).
static int fbb_lanes(int64_t nvals, int64_t n, int B) {
  const double nb = n ? (double)nvals / ((double)n * B) : 0.0;
  if (nb <= 2.0) return 2;
  if (nb <= 4.0) return 4;
  return 8;
}

template <class TA, class TX, class TY, int MODE, int B>
static void fbb_launch(int L, int64_t nbr, hipStream_t st, const int64_t* optr, const int32_t* ocol, const TA* ov,
                       const TX* x, const TY* b, TY omega, TY* y, const int32_t* list, TY* y2, const TX* xc,
                       const int32_t* own) {
#define FBB(LP) hipLaunchKernelGGL((k_fbb<TA, TX, TY, B, LP, MODE>), dim3((unsigned)cdiv(nbr * LP, 256)), dim3(256), 0, \
                                   st, nbr, optr, ocol, ov, x, b, omega, y, list, y2, xc, own)
  switch (L) {
    case 2: FBB(2); break;
    case 4: FBB(4); break;
    default: FBB(8); break;
  }
#undef FBB
}

// k_fbb over n rows (the listed ones for SP_SWEEP_LIST, whole blocks in
// increasing order), block size B, L lanes per block row.
template <class TA, class TX, class TY, int MODE>
static ah_status fbb_g(int B, int L, int64_t n, const int64_t* optr, const int32_t* ocol, const TA* ov, const TX* x,
                       const TY* b, TY omega, TY* y, hipStream_t st, const char* tag = nullptr, double bytes = 0.0,
                       const int32_t* list = nullptr, TY* y2 = nullptr, const TX* xc = nullptr,
                       const int32_t* own = nullptr) {
  if (n == 0) return AH_OK;
  if (n % B) { set_error("block-row sweep over %lld rows, not whole blocks of %d", (long long)n, B); return AH_EINVAL; }
  const int64_t nbr = n / B;
  ProfScope ps;
  prof_begin(ps, tag, st, bytes);
  switch (B) {
    case 2: fbb_launch<TA, TX, TY, MODE, 2>(L, nbr, st, optr, ocol, ov, x, b, omega, y, list, y2, xc, own); break;
    case 3: fbb_launch<TA, TX, TY, MODE, 3>(L, nbr, st, optr, ocol, ov, x, b, omega, y, list, y2, xc, own); break;
    case 4: fbb_launch<TA, TX, TY, MODE, 4>(L, nbr, st, optr, ocol, ov, x, b, omega, y, list, y2, xc, own); break;
    case 6: fbb_launch<TA, TX, TY, MODE, 6>(L, nbr, st, optr, ocol, ov, x, b, omega, y, list, y2, xc, own); break;
    case 10: fbb_launch<TA, TX, TY, MODE, 10>(L, nbr, st, optr, ocol, ov, x, b, omega, y, list, y2, xc, own); break;
    default: set_error("unsupported facet block size %d", B); return AH_EUNSUPPORTED;
  }
  prof_end(ps);
  AH_LAUNCHED();
  return AH_OK;
}

// Level-0 kernel over n rows of the facet-block layout: by block rows
// (k_fbb) where the rows are whole blocks (all rows, or block AIR point
// lists), else by rows (k_fb).
template <class T, int MODE>
static ah_status fb_any(const ah_hier* h, const AhLevel& L, bool blocks, int64_t n, const T* ov, const T* x,
                        const T* b, T om, T* y, hipStream_t st, const char* tag = nullptr, double bytes = 0.0,
                        const int32_t* list = nullptr, T* y2 = nullptr) {
  if (blocks && h->fbb) {
    const int lp = h->lpb ? h->lpb : fbb_lanes(L.nov, L.n, L.ob);
    return fbb_g<T, T, T, MODE>(L.ob, lp, n, L.optr, L.ocol, ov, x, b, om, y, st, tag, bytes, list, y2);
  }
  const int Gb = h->g0 ? h->g0 : fb_lanes(L.nov, L.n);
  return fb_g<T, T, T, MODE>(L.ob, Gb, n, L.optr, L.ocol, ov, x, b, om, y, st, tag, bytes, list, y2);
}

// Algorithmic bytes of a Jacobi sweep on the point set X of level L: the X
// rows of A once, x once, b and d on X, the X updates written.
template <class T>
static double sweep_bytes(const AhLevel& L, int X) {
  const double w = sizeof(T);
  const int64_t nX = X == 0 ? L.nF : L.n - L.nF;
  const int64_t nnzX = X == 0 ? L.nnzF : L.nnz - L.nnzF;
  return (double)nnzX * (w + 4.0) + (double)(nX + 1) * 8.0 + (double)L.n * w + (double)nX * 3.0 * w;
}

// The same for a level-0 sweep in the off-diagonal facet-block layout: the
// X rows' values, every block column index and block-row offset, the list,
// x once, b on X, the X updates written (twice with a second output).
// With xc (the sweeps reading P e_c from e_c): the iterate read once is e_c
// (first F sweep) or x on F and e_c on C, and the first F sweep reads the
// F blocks' coarse blocks under P.
template <class T>
static double fb_sweep_bytes(const AhLevel& L, int X, bool y2, int xc = 0) {
  const double w = sizeof(T);
  const int64_t nX = X == 0 ? L.nF : L.n - L.nF;
  const int64_t nvX = X == 0 ? L.novF : L.nov - L.novF;
  const double xonce = xc == 1 ? (double)L.nc * w : (double)L.n * w;
  const double own = xc == 1 ? (double)(nX / L.ob) * 4.0 : 0.0;
  return (double)nvX * w + (double)(L.nov / (L.ob * L.ob)) * 4.0 + (double)(L.n / L.ob + 1) * 8.0 +
         (double)nX * 4.0 + xonce + own + (double)nX * (y2 ? 3.0 : 2.0) * w;
}

// The same for a sweep of a coarse level read by full blocks: the X rows'
// values, every block column index, the block-row offsets and value bases
// (or, from the copy in sweep order, the X rows' 16-byte records), the list,
// x once, b and d on X, the X updates written (twice with a second output).
template <class T>
static double fbr_sweep_bytes(const AhLevel& L, int X, bool y2) {
  const double w = sizeof(T);
  const int64_t nX = X == 0 ? L.nF : L.n - L.nF;
  const int64_t nvX = X == 0 ? L.nbvF : L.nbv - L.nbvF;
  const double rows = L.bsrec ? (double)nX * 16.0 : (double)(L.n / L.bb) * 16.0 + 8.0;
  return (double)nvX * w + (double)(L.nbv / (L.bb * L.bb)) * 4.0 + rows + (double)nX * 4.0 + (double)L.n * w +
         (double)nX * (y2 ? 4.0 : 3.0) * w;
}

// Algorithmic bytes of the block restriction: Z's values, one column index
// per block, the coarse-block offsets, the fine list, x on the neighbourhood
// blocks and the own blocks once (at most all of x), the coarse vector
// written.
template <class T>
static double rz_bytes(const AhLevel& L) {
  const double w = sizeof(T);
  const int64_t nblk = L.nrz / ((int64_t)L.ob * L.ob);
  return (double)L.nrz * w + (double)nblk * 4.0 + (double)(L.nc / L.ob + 1) * 8.0 + (double)L.nc * 4.0 +
         (double)L.n * w + (double)L.nc * w;
}

ah_status tail_image_build(ah_hier* h, hipStream_t st) {
  if (!h->tail_lds || h->tail0 < 0) return AH_OK;
  const int nlev = (int)h->lev.size();
  for (int w = 0; w < 2; ++w) {
    if (w == 1 && !h->prm.fp32_cycle) break;
    double* img = nullptr;
    AH_TRY(h->arena.get(&img, (h->tail_bytes[w] + 15) / 8 + 2));
    if (w == 0)
      hipLaunchKernelGGL(k_tail_image<double>, dim3(1), dim3(1024), 0, st, h->d_tail, h->tail0, nlev, h->cinv,
                         reinterpret_cast<char*>(img));
    else
      hipLaunchKernelGGL(k_tail_image<float>, dim3(1), dim3(1024), 0, st, h->d_tail, h->tail0, nlev, h->cinv,
                         reinterpret_cast<char*>(img));
    AH_LAUNCHED();
    h->tail_img[w] = reinterpret_cast<const char*>(img);
  }
  if (h->tail_lds_t) {
    for (int w = 0; w < 2; ++w) {
      if (w == 1 && !h->prm.fp32_cycle) break;
      double* img = nullptr;
      AH_TRY(h->arena.get(&img, (h->tail_bytes_t[w] + 15) / 8 + 2));
      if (w == 0)
        hipLaunchKernelGGL(k_tail_image_t<double>, dim3(1), dim3(1024), 0, st, h->d_tail, h->tail0, nlev, h->cinv,
                           reinterpret_cast<char*>(img));
      else
        hipLaunchKernelGGL(k_tail_image_t<float>, dim3(1), dim3(1024), 0, st, h->d_tail, h->tail0, nlev, h->cinv,
                           reinterpret_cast<char*>(img));
      AH_LAUNCHED();
      h->tail_img_t[w] = reinterpret_cast<const char*>(img);
    }
  }
  return AH_OK;
}

// ------------------------------------------------------------ V-cycles
template <class T>
struct Ops;
template <>
struct Ops<double> {
  static const double* A(const AhLevel& L) { return L.val; }
  static const double* AT(const AhLevel& L) { return L.ATval; }
  static const double* R(const AhLevel& L) { return L.Rval; }
  static const double* RT(const AhLevel& L) { return L.RTval; }
  static const double* d(const AhLevel& L) { return L.diag; }
  static const double* O(const AhLevel& L) { return L.oval; }
  static const double* OT(const AhLevel& L) { return L.otval; }
  static const double* BX(const AhLevel& L) { return L.baux; }
  static const double* SO(const AhLevel& L) { return L.soval; }
  static const double* CO(const AhLevel& L) { return L.coval; }
  static const double* RZ(const AhLevel& L) { return L.rzval; }
  static double* b(AhLevel& L) { return L.b; }
  static double* x(AhLevel& L) { return L.x; }
  static double* y(AhLevel& L) { return L.y; }
  static double* e(AhLevel& L) { return L.e; }
};
template <>
struct Ops<float> {
  static const float* A(const AhLevel& L) { return L.val32; }
  static const float* AT(const AhLevel& L) { return L.ATval32; }
  static const float* R(const AhLevel& L) { return L.Rval32; }
  static const float* RT(const AhLevel& L) { return L.RTval32; }
  static const float* d(const AhLevel& L) { return L.diag32; }
  static const float* O(const AhLevel& L) { return L.oval32; }
  static const float* OT(const AhLevel& L) { return L.otval32; }
  static const float* BX(const AhLevel& L) { return L.baux32; }
  static const float* SO(const AhLevel& L) { return L.soval32; }
  static const float* CO(const AhLevel& L) { return L.coval32; }
  static const float* RZ(const AhLevel& L) { return L.rzval32; }
  static float* b(AhLevel& L) { return L.b32; }
  static float* x(AhLevel& L) { return L.x32; }
  static float* y(AhLevel& L) { return L.y32; }
  static float* e(AhLevel& L) { return L.e32; }
};

// Ordered sweeps on level 0 (relax 2: all points; relax 3: F points, then
// all points), one launch per level of the flow order, from xo into xn
// (xn must hold the same values as xo on entry).
template <class TA, class T, int B, int G>
static void gs_fb_level(bool blk, int64_t nrows, const int4* rec, const ah_hier* h, const TA* ov, const T* b,
                        const T* xo, T* xn, hipStream_t st) {
  const dim3 grid((unsigned)cdiv(nrows * G, 256));
  if (blk)
    hipLaunchKernelGGL((k_gs_fb<TA, T, B, G, true>), grid, dim3(256), 0, st, nrows, rec, h->ord_cols, ov, b, xo, xn);
  else
    hipLaunchKernelGGL((k_gs_fb<TA, T, B, G, false>), grid, dim3(256), 0, st, nrows, rec, h->ord_cols, ov, b, xo, xn);
}

template <class T, int B>
static ah_status gs_fb_sweep_b(const ah_hier* h, bool fonly, const T* ov, const T* b, const T* xo, T* xn,
                               hipStream_t st) {
  const AhLevel& L = h->lev[0];
  const int G = fb_lanes(L.nov, L.n) <= 4 ? 4 : 8;
  const std::vector<int64_t>& lp = fonly ? h->ord_lptrF : h->ord_lptr;
  const int64_t scale = fonly ? 1 : B;
  const int4* rec = fonly ? h->ord_finfo : h->ord_info;
  for (size_t k = 0; k + 1 < lp.size(); ++k) {
    const int64_t nr = (lp[k + 1] - lp[k]) * scale;
    if (nr == 0) continue;
    if (G == 4)
      gs_fb_level<T, T, B, 4>(!fonly, nr, rec + lp[k], h, ov, b, xo, xn, st);
    else
      gs_fb_level<T, T, B, 8>(!fonly, nr, rec + lp[k], h, ov, b, xo, xn, st);
  }
  AH_LAUNCHED();
  return AH_OK;
}

// Algorithmic bytes of one ordered sweep: the swept rows of A once (values,
// one column index per block, block offsets), x once, b read and the rows
// written, the item lists.
template <class T>
static double gs_sweep_bytes(const AhLevel& L, bool fonly) {
  const double w = sizeof(T);
  const int64_t nX = fonly ? L.nF : L.n;
  const int64_t nvX = fonly ? L.novF : L.nov;
  return (double)nvX * w + (double)(L.nov / (L.ob * L.ob)) * 4.0 + (double)(L.n / L.ob + 1) * 8.0 +
         (double)L.n * w + (double)nX * 2.0 * w + (double)(fonly ? nX : L.n / L.ob) * 4.0;
}

template <class T>
static ah_status gs_fb_sweep(const ah_hier* h, bool fonly, const T* ov, const T* b, const T* xo, T* xn,
                             hipStream_t st) {
  const AhLevel& L = h->lev[0];
  ProfScope ps;
  prof_begin(ps, fonly ? (sizeof(T) == 8 ? "gs0_f" : "gs0_f_f32") : (sizeof(T) == 8 ? "gs0" : "gs0_f32"), st,
             gs_sweep_bytes<T>(L, fonly));
  ah_status rc = AH_OK;
  switch (L.ob) {
    case 2: rc = gs_fb_sweep_b<T, 2>(h, fonly, ov, b, xo, xn, st); break;
    case 3: rc = gs_fb_sweep_b<T, 3>(h, fonly, ov, b, xo, xn, st); break;
    case 4: rc = gs_fb_sweep_b<T, 4>(h, fonly, ov, b, xo, xn, st); break;
    case 6: rc = gs_fb_sweep_b<T, 6>(h, fonly, ov, b, xo, xn, st); break;
    case 10: rc = gs_fb_sweep_b<T, 10>(h, fonly, ov, b, xo, xn, st); break;
    default: set_error("unsupported facet block size %d", L.ob); rc = AH_EUNSUPPORTED;
  }
  prof_end(ps);
  return rc;
}

// Transposed ordered sweep on the rows of A_0^T, levels in reverse order,
// from yo into yn (equal on entry).
template <class T>
static ah_status gs_csr_sweep_t(const ah_hier* h, bool fonly, const T* atv, const T* d, const T* g, const T* yo,
                                T* yn, hipStream_t st) {
  const AhLevel& L = h->lev[0];
  const std::vector<int64_t>& lp = fonly ? h->ord_lptrF : h->ord_lptr;
  const int B = L.ob;
  const int64_t scale = fonly ? 1 : B;
  const int32_t* items = fonly ? h->ord_frows : h->ord;
  if (lp.size() < 2) return AH_OK;
  for (size_t k = lp.size() - 1; k-- > 0;) {
    const int64_t nr = (lp[k + 1] - lp[k]) * scale;
    if (nr == 0) continue;
    const dim3 grid((unsigned)cdiv(nr * 8, 256));
    if (fonly)
      hipLaunchKernelGGL((k_gs_csr<T, 8, false>), grid, dim3(256), 0, st, nr, items + lp[k], B, L.ATptr, L.ATcol,
                         atv, d, g, h->ord_level, (int)k, yo, yn);
    else
      hipLaunchKernelGGL((k_gs_csr<T, 8, true>), grid, dim3(256), 0, st, nr, items + lp[k], B, L.ATptr, L.ATcol,
                         atv, d, g, h->ord_level, (int)k, yo, yn);
  }
  AH_LAUNCHED();
  return AH_OK;
}

// Forward cycle on level l: b -> out.  out must differ from b and from the
// level's sweep buffers x and y (the second F sweep writes its rows into out
// while other rows still read y): callers pass the level's e buffer or an
// external vector.  The recursion writes the coarse correction into the
// coarse level's e.
template <class T>
static ah_status vcycle(ah_hier* h, int l, const T* b, T* out, hipStream_t st) {
  AhLevel& L = h->lev[l];
  const int nlev = (int)h->lev.size();
  const int nsw = h->prm.relax == 1 ? 1 : 3;
  if (h->tail0 >= 0 && l >= h->tail0) {
    if (h->tail_lds) {
      static std::once_flag once;
      std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void*)k_tail_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)TAIL_LDS_MAX);
        (void)hipFuncSetAttribute((const void*)k_tail_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)TAIL_LDS_MAX);
      });
      const int64_t bytes = h->tail_bytes[sizeof(T) == 8 ? 0 : 1];
      hipLaunchKernelGGL((k_tail_lds<T>), dim3(1), dim3(1024), (unsigned)bytes, st, h->d_tail, l, nlev,
                         h->tail_img[sizeof(T) == 8 ? 0 : 1], b, out, nsw, (T)h->prm.omega);
    } else {
      hipLaunchKernelGGL((k_tail<T, false>), dim3(1), dim3(1024), 0, st, h->d_tail, l, nlev, h->cinv, b, out, nsw,
                         (T)h->prm.omega);
    }
    AH_LAUNCHED();
    return AH_OK;
  }
  if (l == nlev - 1) {
    if (L.n == 0) return AH_OK;
    hipLaunchKernelGGL(k_coarse<T>, dim3((unsigned)L.n), dim3(64), 0, st, (int)L.n, h->cinv, b, out, 0);
    AH_LAUNCHED();
    return AH_OK;
  }
  AhLevel& C = h->lev[l + 1];
  const int G = (l == 0 && h->g0) ? h->g0 : (l > 0 && h->gc) ? h->gc : pick_g(L.nnz, L.n);
  const int GR = pick_g(L.nnzR, L.nc);
  if (l == 0 && L.rzptr && Ops<T>::RZ(L)) {
    // block AIR: R = [Z I] by coarse blocks
    const int lp = fbb_lanes(L.nrz, L.nc, L.ob);
    AH_TRY((fbb_g<T, T, T, SP_RESTRICT>(L.ob, lp, L.nc, L.rzptr, L.rzcol, Ops<T>::RZ(L), b, (const T*)nullptr, (T)0,
                                        Ops<T>::b(C), st, sizeof(T) == 8 ? "restrict0" : "restrict0_f32",
                                        rz_bytes<T>(L), L.clist)));
  } else {
    AH_TRY((csr_g<T, T, T, SP_MV>(GR, L.nc, L.Rptr, L.Rcol, Ops<T>::R(L), b, (const T*)nullptr, (const T*)nullptr,
                                  (const int8_t*)nullptr, 0, (T)0, Ops<T>::b(C), st)));
  }
  T* ec = Ops<T>::e(C);
  AH_TRY(vcycle<T>(h, l + 1, Ops<T>::b(C), ec, st));
  const T om = (T)h->prm.omega;
  const int64_t nF = L.n - L.nc;
  if (l > 0 && L.n < h->list_min) {
    // small coarse levels (launch-latency bound): the first F sweep reads
    // P e_c through pcol and writes every row of y (C rows: P e_c); the
    // second F sweep writes every row of x and its F rows into out; the C
    // sweep visits the C points from their list and writes them into out
    if (nsw == 1) {
      AH_TRY((csr_g<T, T, T, SP_SWEEP_P>(G, L.n, L.rowptr, L.col, Ops<T>::A(L), ec, b, Ops<T>::d(L), L.cf, 0, om,
                                         out, st, nullptr, 0.0, L.pcol)));
      return AH_OK;
    }
    T* x = Ops<T>::x(L);
    T* y = Ops<T>::y(L);
    AH_TRY((csr_g<T, T, T, SP_SWEEP_P>(G, L.n, L.rowptr, L.col, Ops<T>::A(L), ec, b, Ops<T>::d(L), L.cf, 0, om, y,
                                       st, nullptr, 0.0, L.pcol)));
    AH_TRY((csr_g<T, T, T, SP_SWEEP>(G, L.n, L.rowptr, L.col, Ops<T>::A(L), y, b, Ops<T>::d(L), L.cf, 0, om, x, st,
                                     nullptr, 0.0, nullptr, out)));
    AH_TRY((csr_g<T, T, T, SP_SWEEP_LIST>(G, L.nc, L.rowptr, L.col, Ops<T>::A(L), x, b, Ops<T>::d(L), L.cf, 1, om,
                                          out, st, nullptr, 0.0, L.clist)));
    return AH_OK;
  }
  // level 0 and large coarse levels (bandwidth bound): x = y = P e_c, then
  // the F sweeps visit the F points only (from the F list) and the C sweep
  // the C points only, so the C entries of x and y keep the interpolated
  // values through the F sweeps: F1 x -> y, F2 y -> x (its rows also written
  // into out), C x -> out.  With one F sweep, y is out.
  if (l == 0 && h->prm.relax >= 2) {
    // ordered sweeps in the flow order: y = out = P e_c; (relax 3: F sweep
    // y -> out, y = out;) sweep over all points y -> out
    T* y = Ops<T>::y(L);
    hipLaunchKernelGGL((k_interp2<T>), g1(L.n), dim3(256), 0, st, L.n, L.pcol, ec, y, out);
    AH_LAUNCHED();
    const T* ov = Ops<T>::O(L);
    if (h->prm.relax == 3) {
      AH_TRY(gs_fb_sweep<T>(h, true, ov, b, y, out, st));
      AH_HIP(hipMemcpyAsync(y, out, L.n * sizeof(T), hipMemcpyDeviceToDevice, st));
    }
    return gs_fb_sweep<T>(h, false, ov, b, y, out, st);
  }
  T* x = Ops<T>::x(L);
  T* y = nsw == 1 ? out : Ops<T>::y(L);
  // block AIR on level 0 with the encoded copy: the sweeps read P e_c from
  // e_c, so P e_c is never formed
  const bool pfree = l == 0 && nsw == 3 && L.sperm && L.soce && Ops<T>::SO(L);
  if (!pfree) {
    hipLaunchKernelGGL((k_interp2<T>), g1(L.n), dim3(256), 0, st, L.n, L.pcol, ec, x, y);
    AH_LAUNCHED();
  }
  // level-0 timing tags, and level 1's where it is read by full blocks
  const bool t1 = l == 1 && L.bb;
  const char* tf = l == 0 ? (sizeof(T) == 8 ? "relax0_f" : "relax0_f_f32")
                   : t1 ? (sizeof(T) == 8 ? "relax1_f" : "relax1_f_f32") : nullptr;
  const char* tc = l == 0 ? (sizeof(T) == 8 ? "relax0_c" : "relax0_c_f32")
                   : t1 ? (sizeof(T) == 8 ? "relax1_c" : "relax1_c_f32") : nullptr;
  if (l == 0 && L.sperm && Ops<T>::SO(L)) {
    // block AIR with the sweep-ordered copy: the F blocks, then the C
    // blocks, each set one contiguous range of block rows
    const T* so = Ops<T>::SO(L);
    const int lp = h->lpb ? h->lpb : fbb_lanes(L.nov, L.n, L.ob);
    const int64_t nbF = nF / L.ob;
    if (pfree) {
      // F1: P e_c -> y; F2: y on F, e_c on C -> x and out; C: x on F, e_c on C -> out
      AH_TRY((fbb_g<T, T, T, SP_SO_P>(L.ob, lp, nF, L.soptr, L.socp, so, ec, b, om, y, st, tf,
                                      fb_sweep_bytes<T>(L, 0, false, 1), L.sperm, nullptr, ec, L.soown)));
      AH_TRY((fbb_g<T, T, T, SP_SO_E>(L.ob, lp, nF, L.soptr, L.soce, so, y, b, om, x, st, tf,
                                      fb_sweep_bytes<T>(L, 0, true, 2), L.sperm, out, ec, nullptr)));
      AH_TRY((fbb_g<T, T, T, SP_SO_C>(L.ob, lp, L.nc, L.soptr + nbF, L.soce, so, x, b, om, out, st, tc,
                                      fb_sweep_bytes<T>(L, 1, false, 2), L.sperm + nbF, nullptr, ec)));
      return AH_OK;
    }
    AH_TRY((fbb_g<T, T, T, SP_SWEEP_ORD>(L.ob, lp, nF, L.soptr, L.socol, so, x, b, om, y, st, tf,
                                         fb_sweep_bytes<T>(L, 0, false), L.sperm)));
    if (nsw == 1) return AH_OK;
    AH_TRY((fbb_g<T, T, T, SP_SWEEP_ORD>(L.ob, lp, nF, L.soptr, L.socol, so, y, b, om, x, st, tf,
                                         fb_sweep_bytes<T>(L, 0, true), L.sperm, out)));
    AH_TRY((fbb_g<T, T, T, SP_SWEEP_ORD>(L.ob, lp, L.nc, L.soptr + nbF, L.socol, so, x, b, om, out, st, tc,
                                         fb_sweep_bytes<T>(L, 1, false), L.sperm + nbF)));
    return AH_OK;
  }
  if (l == 0 && !L.fblk && L.rsoff && Ops<T>::SO(L)) {
    // scalar AIR: the rows' values in sweep order (the F rows, then the C rows)
    const T* so = Ops<T>::SO(L);
    const int Gb = h->g0 ? h->g0 : fb_lanes(L.nov, L.n);
    AH_TRY((fb_g<T, T, T, SP_SWEEP_ORD>(L.ob, Gb, nF, L.optr, L.ocol, so, x, b, om, y, st, tf,
                                        fb_sweep_bytes<T>(L, 0, false), L.flist, nullptr, L.rsoff)));
    if (nsw == 1) return AH_OK;
    AH_TRY((fb_g<T, T, T, SP_SWEEP_ORD>(L.ob, Gb, nF, L.optr, L.ocol, so, y, b, om, x, st, tf,
                                        fb_sweep_bytes<T>(L, 0, true), L.flist, out, L.rsoff)));
    AH_TRY((fb_g<T, T, T, SP_SWEEP_ORD>(L.ob, Gb, L.nc, L.optr, L.ocol, so, x, b, om, out, st, tc,
                                        fb_sweep_bytes<T>(L, 1, false), L.clist, nullptr, L.rsoff + nF)));
    return AH_OK;
  }
  if (l == 0 && L.ob && Ops<T>::O(L)) {
    const T* ov = Ops<T>::O(L);
    AH_TRY((fb_any<T, SP_SWEEP_LIST>(h, L, L.fblk, nF, ov, x, b, om, y, st, tf, fb_sweep_bytes<T>(L, 0, false),
                                     L.flist)));
    if (nsw == 1) return AH_OK;
    AH_TRY((fb_any<T, SP_SWEEP_LIST>(h, L, L.fblk, nF, ov, y, b, om, x, st, tf, fb_sweep_bytes<T>(L, 0, true),
                                     L.flist, out)));
    AH_TRY((fb_any<T, SP_SWEEP_LIST>(h, L, L.fblk, L.nc, ov, x, b, om, out, st, tc, fb_sweep_bytes<T>(L, 1, false),
                                     L.clist)));
    return AH_OK;
  }
  if (l > 0 && L.bb && Ops<T>::A(L) && Ops<T>::BX(L)) {
    // level 1 under block AIR: the sweeps read it by full blocks
    const T* av = Ops<T>::A(L);
    const T* ax = Ops<T>::BX(L);
    const T* d = Ops<T>::d(L);
    if (Ops<T>::SO(L) && L.bsrec) {
      // from the copy in sweep order: the F rows, then the C rows
      const T* so = Ops<T>::SO(L);
      AH_TRY(fbr_g<T>(L, so, so, nF, L.flist, x, b, d, om, y, st, tf, fbr_sweep_bytes<T>(L, 0, false), nullptr,
                      L.bsrec));
      if (nsw == 1) return AH_OK;
      AH_TRY(fbr_g<T>(L, so, so, nF, L.flist, y, b, d, om, x, st, tf, fbr_sweep_bytes<T>(L, 0, true), out,
                      L.bsrec));
      AH_TRY(fbr_g<T>(L, so, so, L.nc, L.clist, x, b, d, om, out, st, tc, fbr_sweep_bytes<T>(L, 1, false), nullptr,
                      L.bsrec + nF));
      return AH_OK;
    }
    AH_TRY(fbr_g<T>(L, av, ax, nF, L.flist, x, b, d, om, y, st, tf, fbr_sweep_bytes<T>(L, 0, false)));
    if (nsw == 1) return AH_OK;
    AH_TRY(fbr_g<T>(L, av, ax, nF, L.flist, y, b, d, om, x, st, tf, fbr_sweep_bytes<T>(L, 0, true), out));
    AH_TRY(fbr_g<T>(L, av, ax, L.nc, L.clist, x, b, d, om, out, st, tc, fbr_sweep_bytes<T>(L, 1, false)));
    return AH_OK;
  }
  if (l > 0 && L.coptr && Ops<T>::CO(L)) {
    // the rows' entries in sweep order: the F rows, then the C rows
    const T* co = Ops<T>::CO(L);
    const T* d = Ops<T>::d(L);
    AH_TRY((csr_g<T, T, T, SP_SWEEP_ORD>(G, nF, L.coptr, L.cocol, co, x, b, d, L.cf, 0, om, y, st, tf,
                                         sweep_bytes<T>(L, 0), L.flist)));
    if (nsw == 1) return AH_OK;
    AH_TRY((csr_g<T, T, T, SP_SWEEP_ORD>(G, nF, L.coptr, L.cocol, co, y, b, d, L.cf, 0, om, x, st, tf,
                                         sweep_bytes<T>(L, 0), L.flist, out)));
    AH_TRY((csr_g<T, T, T, SP_SWEEP_ORD>(G, L.nc, L.coptr + nF, L.cocol, co, x, b, d, L.cf, 1, om, out, st, tc,
                                         sweep_bytes<T>(L, 1), L.clist)));
    return AH_OK;
  }
  AH_TRY((csr_g<T, T, T, SP_SWEEP_LIST>(G, nF, L.rowptr, L.col, Ops<T>::A(L), x, b, Ops<T>::d(L), L.cf, 0, om, y,
                                        st, tf, sweep_bytes<T>(L, 0), L.flist)));
  if (nsw == 1) return AH_OK;
  AH_TRY((csr_g<T, T, T, SP_SWEEP_LIST>(G, nF, L.rowptr, L.col, Ops<T>::A(L), y, b, Ops<T>::d(L), L.cf, 0, om, x,
                                        st, tf, sweep_bytes<T>(L, 0), L.flist, out)));
  AH_TRY((csr_g<T, T, T, SP_SWEEP_LIST>(G, L.nc, L.rowptr, L.col, Ops<T>::A(L), x, b, Ops<T>::d(L), L.cf, 1, om,
                                        out, st, tc, sweep_bytes<T>(L, 1), L.clist)));
  return AH_OK;
}

// Transposed cycle on level l: g -> out (out may alias g, not the level's
// x or y).  The recursion writes its result over the coarse level's input
// (or into the coarsest level's x).
template <class T>
static ah_status vcycle_t(ah_hier* h, int l, const T* g, T* out, hipStream_t st) {
  AhLevel& L = h->lev[l];
  const int nlev = (int)h->lev.size();
  if (h->tail0 >= 0 && l >= h->tail0) {
    if (h->tail_lds_t && l == h->tail0) {
      static std::once_flag once;
      std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void*)k_tail_lds_t<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)TAIL_LDS_MAX);
        (void)hipFuncSetAttribute((const void*)k_tail_lds_t<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)TAIL_LDS_MAX);
      });
      const int64_t bytes = h->tail_bytes_t[sizeof(T) == 8 ? 0 : 1];
      hipLaunchKernelGGL((k_tail_lds_t<T>), dim3(1), dim3(1024), (unsigned)bytes, st, h->d_tail, l, nlev,
                         h->tail_img_t[sizeof(T) == 8 ? 0 : 1], g, out, h->prm.relax == 1 ? 1 : 3,
                         (T)h->prm.omega);
    } else {
      hipLaunchKernelGGL((k_tail<T, true>), dim3(1), dim3(1024), 0, st, h->d_tail, l, nlev, h->cinv, g, out,
                         h->prm.relax == 1 ? 1 : 3, (T)h->prm.omega);
    }
    AH_LAUNCHED();
    return AH_OK;
  }
  if (l == nlev - 1) {
    if (L.n == 0) return AH_OK;
    hipLaunchKernelGGL(k_coarse<T>, dim3((unsigned)L.n), dim3(64), 0, st, (int)L.n, h->cinv, g, out, 1);
    AH_LAUNCHED();
    return AH_OK;
  }
  AhLevel& C = h->lev[l + 1];
  const int G = pick_g(L.nnz, L.n);
  const T om = (T)h->prm.omega;
  T* cur = Ops<T>::x(L);
  T* alt = Ops<T>::y(L);
  const bool fbt = l == 0 && h->prm.relax < 2 && Ops<T>::OT(L);
  if (l == 0 && h->prm.relax >= 2) {
    AH_HIP(hipMemsetAsync(cur, 0, L.n * sizeof(T), st));
    // transposed ordered sweeps: all points, then (relax 3) F points
    AH_HIP(hipMemsetAsync(alt, 0, L.n * sizeof(T), st));
    AH_TRY(gs_csr_sweep_t<T>(h, false, Ops<T>::AT(L), Ops<T>::d(L), g, cur, alt, st));
    std::swap(cur, alt);
    if (h->prm.relax == 3) {
      AH_HIP(hipMemcpyAsync(alt, cur, L.n * sizeof(T), hipMemcpyDeviceToDevice, st));
      AH_TRY(gs_csr_sweep_t<T>(h, true, Ops<T>::AT(L), Ops<T>::d(L), g, cur, alt, st));
      std::swap(cur, alt);
    }
  } else if (fbt) {
    // A_0^T by facet blocks: the first sweep (C points, or the F points
    // with one sweep) starts from zero, y_X = omega g_X / d_X, written to
    // both buffers; the F sweeps then alternate over the F list
    const int X = h->prm.relax == 1 ? 0 : 1;
    hipLaunchKernelGGL((k_sweep_from_zero<T>), g1(L.n), dim3(256), 0, st, L.n, L.cf, X, g, Ops<T>::d(L), om, cur,
                       alt);
    AH_LAUNCHED();
    if (h->prm.relax != 1) {
      AH_TRY((fb_any<T, SP_SWEEP_LIST>(h, L, L.fblk, nF0(L), Ops<T>::OT(L), cur, g, om, alt, st, nullptr, 0.0,
                                       L.flist)));
      AH_TRY((fb_any<T, SP_SWEEP_LIST>(h, L, L.fblk, nF0(L), Ops<T>::OT(L), alt, g, om, cur, st, nullptr, 0.0,
                                       L.flist)));
    }
    // residual g - A^T y, restricted by P^T
    AH_TRY((fb_any<T, SP_RES>(h, L, true, L.n, Ops<T>::OT(L), cur, g, (T)0, alt, st)));
    AH_TRY((csr_g<T, T, T, SP_MV>(4, L.nc, L.PTptr, L.PTcol, (const T*)nullptr, alt, (const T*)nullptr,
                                  (const T*)nullptr, (const int8_t*)nullptr, 0, (T)0, Ops<T>::b(C), st)));
    T* ec = (l + 1 == nlev - 1) ? Ops<T>::x(C) : Ops<T>::b(C);
    AH_TRY(vcycle_t<T>(h, l + 1, Ops<T>::b(C), ec, st));
    const int GR = pick_g(L.nnzR, L.n);
    AH_TRY((csr_g<T, T, T, SP_ADDMV>(GR, L.n, L.RTptr, L.RTcol, Ops<T>::RT(L), ec, cur, (const T*)nullptr,
                                     (const int8_t*)nullptr, 0, (T)0, out, st)));
    return AH_OK;
  } else {
    // the first sweep (C points, or the F points with one sweep) starts from
    // zero, y_X = omega g_X / d_X, written to both buffers; the F sweeps then
    // alternate over the F list
    const int X = h->prm.relax == 1 ? 0 : 1;
    hipLaunchKernelGGL((k_sweep_from_zero<T>), g1(L.n), dim3(256), 0, st, L.n, L.cf, X, g, Ops<T>::d(L), om, cur,
                       alt);
    AH_LAUNCHED();
    if (h->prm.relax != 1) {
      AH_TRY((csr_g<T, T, T, SP_SWEEP_LIST>(G, nF0(L), L.ATptr, L.ATcol, Ops<T>::AT(L), cur, g, Ops<T>::d(L), L.cf, 0,
                                            om, alt, st, nullptr, 0.0, L.flist)));
      AH_TRY((csr_g<T, T, T, SP_SWEEP_LIST>(G, nF0(L), L.ATptr, L.ATcol, Ops<T>::AT(L), alt, g, Ops<T>::d(L), L.cf, 0,
                                            om, cur, st, nullptr, 0.0, L.flist)));
    }
  }
  // residual g - A^T y, restricted by P^T
  AH_TRY((csr_g<T, T, T, SP_RES>(G, L.n, L.ATptr, L.ATcol, Ops<T>::AT(L), cur, g, (const T*)nullptr,
                                 (const int8_t*)nullptr, 0, (T)0, alt, st)));
  AH_TRY((csr_g<T, T, T, SP_MV>(4, L.nc, L.PTptr, L.PTcol, (const T*)nullptr, alt, (const T*)nullptr,
                                (const T*)nullptr, (const int8_t*)nullptr, 0, (T)0, Ops<T>::b(C), st)));
  T* ec = (l + 1 == nlev - 1) ? Ops<T>::x(C) : Ops<T>::b(C);
  AH_TRY(vcycle_t<T>(h, l + 1, Ops<T>::b(C), ec, st));
  // out = y + R^T e_c
  const int GR = pick_g(L.nnzR, L.n);
  AH_TRY((csr_g<T, T, T, SP_ADDMV>(GR, L.n, L.RTptr, L.RTcol, Ops<T>::RT(L), ec, cur, (const T*)nullptr,
                                   (const int8_t*)nullptr, 0, (T)0, out, st)));
  return AH_OK;
}

// Preconditioner application on level 0 for the requested precision:
// r (FP64, level-0 scaled space) -> z (FP64) or z32 (FP32).
static ah_status precond(ah_hier* h, const double* r, double* z, float* z32, int precision, int transpose,
                         hipStream_t st) {
  AhLevel& L = h->lev[0];
  if (precision == 0) {
    return transpose ? vcycle_t<double>(h, 0, r, z, st) : vcycle<double>(h, 0, r, z, st);
  }
  hipLaunchKernelGGL((k_cast<double, float>), g1(L.n), dim3(256), 0, st, L.n, r, L.b32);
  AH_LAUNCHED();
  return transpose ? vcycle_t<float>(h, 0, L.b32, z32, st) : vcycle<float>(h, 0, L.b32, z32, st);
}

// ------------------------------------------------------------ FGMRES
// Workspace of one FGMRES solve: basis V [(m+1)][n], preconditioned vectors
// Z [m][n] (FP64 cycle) or Z32 (FP32 cycle), w, r, the scaled right-hand
// side, the reduction partials [(2m+4)][1024], the device scalars [4 (m+3)]
// and a host staging array of 4 (m+3) doubles for the Hessenberg column.
// air_solve takes it from buffers the hierarchy keeps; air_solve_noalloc
// carves it out of the library's static scratch array.
struct KWork {
  double* V = nullptr;
  double* Z = nullptr;
  float* Z32 = nullptr;
  double* w = nullptr;
  double* r = nullptr;
  double* bhat = nullptr;
  double* partial = nullptr;
  double* hdev = nullptr;
  double* host = nullptr;
};

static ah_status ensure_workspace(ah_hier* h, int m, int precision, hipStream_t st, KWork* W) {
  const int64_t n = h->lev[0].n;
  if (!(h->m_alloc >= m && (precision == 0 ? h->Z != nullptr : h->Z32 != nullptr))) {
    Arena& ar = h->arena;
    ar.stream = st;   // the workspace is allocated on the solving stream
    if (h->m_alloc < m) {
      AH_TRY(ar.get(&h->V, (int64_t)(m + 1) * n));
      AH_TRY(ar.get(&h->w, n));
      AH_TRY(ar.get(&h->r, n));
      AH_TRY(ar.get(&h->bhat, n));
      AH_TRY(ar.get(&h->partial, (int64_t)(2 * m + 4) * 1024));
      AH_TRY(ar.get(&h->hdev, 4 * (m + 3)));
      h->Z = nullptr;
      h->Z32 = nullptr;
      h->m_alloc = m;
    }
    // Z and Z32 hold the full capacity m_alloc (>= m): a later call with a
    // restart up to m_alloc reuses them without a new check
    if (precision == 0 && !h->Z) AH_TRY(ar.get(&h->Z, (int64_t)h->m_alloc * n));
    if (precision == 1 && !h->Z32) AH_TRY(ar.get(&h->Z32, (int64_t)h->m_alloc * n));
  }
  W->V = h->V;
  W->Z = precision == 0 ? h->Z : nullptr;
  W->Z32 = precision == 1 ? h->Z32 : nullptr;
  W->w = h->w;
  W->r = h->r;
  W->bhat = h->bhat;
  W->partial = h->partial;
  W->hdev = h->hdev;
  W->host = pinned_scratch(4 * (m + 3));
  if (!W->host) { set_error("pinned host allocation failed"); return AH_ENOMEM; }
  return AH_OK;
}

// ---------------------------------------------------------- BiCGSTAB
// Device scalars: [0] rho = r_hat.r, [1] r.r, [2] r_hat.v, [3] v.v,
// [4] s.t, [5] t.t, [6] s.s, [7] r.r after the step, [8] rho_old,
// [9] alpha, [10] omega.
enum { BC_RHO = 0, BC_RV = 2, BC_ST = 4, BC_TT = 5, BC_SS = 6, BC_RR = 7, BC_RHOOLD = 8, BC_ALPHA = 9,
       BC_OMEGA = 10, BC_N = 11 };

// p = r + beta (p - omega v), beta = (rho / rho_old) (alpha / omega)
__global__ void k_bicg_p(int64_t n, const double* __restrict__ r, const double* __restrict__ v,
                         double* __restrict__ p, const double* __restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = (sc[BC_RHO] / sc[BC_RHOOLD]) * (sc[BC_ALPHA] / sc[BC_OMEGA]);
  p[i] = r[i] + beta * (p[i] - sc[BC_OMEGA] * v[i]);
}

// alpha = rho / (r_hat.v), s = r - alpha v, block partial sums of s.s
__global__ __launch_bounds__(256) void k_bicg_s(int64_t n, const double* __restrict__ r,
                                                const double* __restrict__ v, double* __restrict__ s,
                                                double* __restrict__ sc, double* __restrict__ partial, int nblk) {
  __shared__ double red[4];
  const double alpha = sc[BC_RHO] / sc[BC_RV];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)nblk * 256) {
    const double si = r[i] - alpha * v[i];
    s[i] = si;
    acc += si * si;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    if (blockIdx.x == 0) sc[BC_ALPHA] = alpha;
  }
}

// x += alpha p_hat (the step ended on s)
__global__ void k_bicg_xhalf(int64_t n, const double* __restrict__ ph, double* __restrict__ x,
                             const double* __restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += sc[BC_ALPHA] * ph[i];
}

// omega = (t.s) / (t.t), x += alpha p_hat + omega s_hat, r = s - omega t,
// block partial sums of r.r; rho_old = rho
__global__ __launch_bounds__(256) void k_bicg_xr(int64_t n, const double* __restrict__ ph,
                                                 const double* __restrict__ sh, const double* __restrict__ s,
                                                 const double* __restrict__ t, double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ sc,
                                                 double* __restrict__ partial, int nblk) {
  __shared__ double red[4];
  const double tt = sc[BC_TT];
  const double omega = tt > 0.0 ? sc[BC_ST] / tt : 0.0;
  const double alpha = sc[BC_ALPHA];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)nblk * 256) {
    x[i] += alpha * ph[i] + omega * sh[i];
    const double ri = s[i] - omega * t[i];
    r[i] = ri;
    acc += ri * ri;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    if (blockIdx.x == 0) {
      sc[BC_OMEGA] = omega;
      sc[BC_RHOOLD] = sc[BC_RHO];
    }
  }
}

// Blocks of the multi-vector dot kernels (at most 1024, about four rows per
// thread).
static int dot_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(n, DOT_T * 4))); }

// out[0..k] = V[0..k-1].w and w.w (k vectors plus the norm), on the device.
static ah_status multidot(int64_t n, int k, const double* V, const double* w, double* partial, double* out,
                          hipStream_t st) {
  int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(n, DOT_T * 4)));
  dim3 grid(nblk, (unsigned)cdiv(k + 1, DOT_V));
  hipLaunchKernelGGL(k_multidot, grid, dim3(DOT_T), 0, st, n, k, V, n, w, partial, nblk);
  AH_LAUNCHED();
  hipLaunchKernelGGL(k_reduce_partial, dim3(k + 1), dim3(256), 0, st, nblk, partial, out, 0);
  AH_LAUNCHED();
  return AH_OK;
}

// Level-0 operator of a Krylov solve: scalar CSR, and for a scaled system's
// forward operator also the off-diagonal facet-block layout (ob > 0), which
// is then the one applied.
struct Op {
  const int64_t* rp;
  const int32_t* ci;
  const double* v;
  int ob = 0;
  const int64_t* optr = nullptr;
  const int32_t* ocol = nullptr;
  const double* ov = nullptr;
  int64_t nov = 0;
  int lpb = 0;                 // > 0: the facet-block layout by block rows (k_fbb), that many lanes each
};

static int op_lanes(const ah_hier* h, const Op& A, int64_t n) {
  if (h->g0) return h->g0;
  return A.ob ? fb_lanes(A.nov, n) : pick_g(h->lev[0].nnz, n);
}

// Algorithmic bytes of y = A x (x of width wx): the operator once, x once,
// y written.
static double op_mv_bytes(const ah_hier* h, const Op& A, int64_t n, double wx) {
  if (A.ob) return (double)A.nov * 8.0 + (double)(A.nov / (A.ob * A.ob)) * 4.0 + (double)(n / A.ob + 1) * 8.0 +
                   (double)n * wx + (double)n * 8.0;
  return (double)h->lev[0].nnz * 12.0 + (double)(n + 1) * 8.0 + (double)n * wx + (double)n * 8.0;
}

// y = A x (SP_MV) or y = b - A x (SP_RES).
template <class TX, int MODE>
static ah_status op_apply(const Op& A, int G, int64_t n, const TX* x, const double* b, double* y, hipStream_t st,
                          const char* tag = nullptr, double bytes = 0.0) {
  if (A.ob && A.lpb)
    return fbb_g<double, TX, double, MODE>(A.ob, A.lpb, n, A.optr, A.ocol, A.ov, x, b, 0.0, y, st, tag, bytes);
  if (A.ob)
    return fb_g<double, TX, double, MODE>(A.ob, G, n, A.optr, A.ocol, A.ov, x, b, 0.0, y, st, tag, bytes);
  return csr_g<double, TX, double, MODE>(G, n, A.rp, A.ci, A.v, x, b, (const double*)nullptr,
                                         (const int8_t*)nullptr, 0, 0.0, y, st, tag, bytes);
}

static ah_status fgmres_dcgs2(ah_hier* h, const KWork& W, Op A, const double* bvec, double* x,
                              const ah_solve_params& prm, int transpose, hipStream_t st, ah_solve_info* info);

static ah_status fgmres(ah_hier* h, const KWork& W, Op A, const double* bvec, double* x, const ah_solve_params& prm,
                        int transpose, hipStream_t st, ah_solve_info* info) {
  const int64_t n = h->lev[0].n;
  if (n >= h->dcgs_min) return fgmres_dcgs2(h, W, A, bvec, x, prm, transpose, st, info);
  const int m = std::max(1, prm.restart);
  const int G0 = op_lanes(h, A, n);
  double* hd = W.hdev;
  double* hh = W.host;
  auto t0 = std::chrono::steady_clock::now();
  // ||b||
  AH_TRY(multidot(n, 0, W.V, bvec, W.partial, hd, st));
  AH_HIP(hipMemcpyAsync(hh, hd, sizeof(double), hipMemcpyDeviceToHost, st));
  AH_HIP(hipStreamSynchronize(st));
  const double bnorm = std::sqrt(hh[0]);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m);
  int its = 0;
  bool converged = false;
  double relres = 1.0, true_rel = 1.0;
  ah_status status = AH_OK;
  if (!(bnorm > 0.0)) {
    AH_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
    if (info) { info->iters = 0; info->converged = 1; info->relres = 0; info->true_relres = 0; }
    return AH_OK;
  }
  if (!std::isfinite(bnorm)) { set_error("air_solve: non-finite right-hand side"); return AH_EBREAKDOWN; }
  while (true) {
    // r = b - A x
    AH_TRY((op_apply<double, SP_RES>(A, G0, n, x, bvec, W.r, st)));
    AH_TRY(multidot(n, 0, W.V, W.r, W.partial, hd, st));
    AH_HIP(hipMemcpyAsync(hh, hd, sizeof(double), hipMemcpyDeviceToHost, st));
    AH_HIP(hipStreamSynchronize(st));
    const double beta = std::sqrt(hh[0]);
    true_rel = beta / bnorm;
    relres = true_rel;
    if (!std::isfinite(beta)) { set_error("air_solve: breakdown (NaN residual)"); status = AH_EBREAKDOWN; break; }
    if (beta <= prm.tol * bnorm) { converged = true; break; }
    if (its >= prm.maxit) break;
    hipLaunchKernelGGL(k_scale, g1(n), dim3(256), 0, st, n, W.r, 1.0 / beta, W.V);
    AH_LAUNCHED();
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int kdone = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = W.V + (int64_t)j * n;
      double* zj = W.Z ? W.Z + (int64_t)j * n : nullptr;
      float* zj32 = W.Z32 ? W.Z32 + (int64_t)j * n : nullptr;
      AH_TRY(precond(h, vj, prm.precision == 0 ? zj : nullptr, prm.precision == 1 ? zj32 : nullptr, prm.precision,
                     transpose, st));
      const double by = op_mv_bytes(h, A, n, prm.precision ? 4.0 : 8.0);
      if (prm.precision == 0)
        AH_TRY((op_apply<double, SP_MV>(A, G0, n, zj, (const double*)nullptr, W.w, st,
                                        transpose ? nullptr : "spmv0", by)));
      else
        AH_TRY((op_apply<float, SP_MV>(A, G0, n, zj32, (const double*)nullptr, W.w, st,
                                       transpose ? nullptr : "spmv0", by)));
      ++its;
      const int k = j + 1;
      // CGS2
      double* h1 = hd;               // [k+1]: dots, then ||w0||^2 at [k]
      double* h2 = hd + (m + 2);     // [k+1]
      double* hn = hd + 2 * (m + 2); // [1]
      // each pass: block partials of the dots, then one kernel that sums
      // them (every block, fixed order) and updates w
      {
        const int nblk = dot_blocks(n);
        const unsigned hb = (unsigned)((k + 1) * sizeof(double));
        double* p3 = W.partial + (int64_t)(m + 2) * 1024;   // clear of the (k+1) nblk dot partials
        hipLaunchKernelGGL(k_multidot, dim3(nblk, (unsigned)cdiv(k + 1, DOT_V)), dim3(DOT_T), 0, st, n, k, W.V, n,
                           W.w, W.partial, nblk);
        hipLaunchKernelGGL(k_maxpy_p, dim3(nblk), dim3(DOT_T), hb, st, n, k, W.V, n, W.partial, nblk, W.w, h1);
        hipLaunchKernelGGL(k_multidot, dim3(nblk, (unsigned)cdiv(k + 1, DOT_V)), dim3(DOT_T), 0, st, n, k, W.V, n,
                           W.w, W.partial, nblk);
        hipLaunchKernelGGL(k_maxpy_norm, dim3(nblk), dim3(DOT_T), hb, st, n, k, W.V, n, W.partial, nblk, W.w, h2,
                           p3);
        hipLaunchKernelGGL(k_reduce_partial, dim3(1), dim3(256), 0, st, nblk, p3, hn, 0);
        AH_LAUNCHED();
      }
      AH_HIP(hipMemcpyAsync(hh, hd, (3 * (m + 2)) * sizeof(double), hipMemcpyDeviceToHost, st));
      AH_HIP(hipStreamSynchronize(st));
      const double w0 = std::sqrt(hh[k]);
      const double hnorm = std::sqrt(hh[2 * (m + 2)]);
      if (!std::isfinite(hnorm) || !std::isfinite(w0)) {
        set_error("air_solve: breakdown (NaN in Arnoldi)");
        status = AH_EBREAKDOWN;
        kdone = j;
        break;
      }
      for (int i = 0; i < k; ++i) H[(size_t)i * m + j] = hh[i] + hh[(m + 2) + i];
      H[(size_t)k * m + j] = hnorm;
      for (int i = 0; i < j; ++i) {
        double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)k * m + j];
      const double den = std::hypot(a, bb);
      if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; } else { cs[j] = a / den; sn[j] = bb / den; }
      H[(size_t)j * m + j] = cs[j] * a + sn[j] * bb;
      H[(size_t)k * m + j] = 0.0;
      g[k] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      kdone = k;
      relres = std::fabs(g[k]) / bnorm;
      const bool happy = hnorm <= 1e-14 * w0;
      if (std::fabs(g[k]) <= prm.tol * bnorm || happy || its >= prm.maxit) break;
      hipLaunchKernelGGL(k_scale, g1(n), dim3(256), 0, st, n, W.w, 1.0 / hnorm, W.V + (int64_t)k * n);
      AH_LAUNCHED();
    }
    if (status != AH_OK && kdone == 0) break;
    for (int i = kdone - 1; i >= 0; --i) {
      double s = g[i];
      for (int c = i + 1; c < kdone; ++c) s -= H[(size_t)i * m + c] * y[c];
      y[i] = s / H[(size_t)i * m + i];
    }
    AH_HIP(hipMemcpyAsync(hd, y.data(), kdone * sizeof(double), hipMemcpyHostToDevice, st));
    if (prm.precision == 0)
      hipLaunchKernelGGL(k_maxpy<double>, g1(n), dim3(256), 0, st, n, kdone, W.Z, n, hd, x, 1.0);
    else
      hipLaunchKernelGGL(k_maxpy<float>, g1(n), dim3(256), 0, st, n, kdone, W.Z32, n, hd, x, 1.0);
    AH_LAUNCHED();
    if (status != AH_OK) break;
  }
  AH_HIP(hipStreamSynchronize(st));
  if (info) {
    info->iters = its;
    info->converged = converged ? 1 : 0;
    info->relres = relres;
    info->true_relres = true_rel;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status != AH_OK) return status;
  return converged ? AH_OK : AH_ENOCONV;
}

// FGMRES with delayed CGS2 orthogonalisation: the basis is read twice per
// iteration instead of four times.  The candidate u_j (w_{j-1} projected
// once, not normalised) is preconditioned and multiplied right away,
// z~_j = M u_j, w_j = A z~_j; one dot pass then gives Q^T u_j, |u_j|^2,
// Q^T w_j and u_j.w_j.  The second projection of u_j finishes it,
// u_j = Q a + r_jj q_j with r_jj = sqrt(|u_j|^2 - |a|^2), and completes
// Hessenberg column j-1 (+a, subdiagonal r_jj).  Since A is linear,
// A z_j = (w_j - A Z a) / r_jj for z_j = (z~_j - Z a) / r_jj, which gives
// column j from the dots and the finished columns, and the next candidate
// u_{j+1} = (w_j - Q c - q_j d) / r_jj, formed in one update pass together
// with q_j.  The solution uses z~ directly: Z~ = Z R with R upper triangular
// (column j = [a; r_jj]), so x += Z~ (R^-1 y).  Convergence of column j-1
// is known one step late, after z~_j and w_j are formed: one extra cycle
// per restart cycle, which is why the plain CGS2 loop is kept for small
// systems.
static ah_status fgmres_dcgs2(ah_hier* h, const KWork& W, Op A, const double* bvec, double* x,
                              const ah_solve_params& prm, int transpose, hipStream_t st, ah_solve_info* info) {
  const int64_t n = h->lev[0].n;
  const int m = std::max(1, prm.restart);
  const int G0 = op_lanes(h, A, n);
  double* hd = W.hdev;
  double* hh = W.host;
  double* coef_d = hd + (2 * m + 3);
  double* coef_h = hh + (2 * m + 3);
  const int nblk = dot_blocks(n);
  auto t0 = std::chrono::steady_clock::now();
  AH_TRY(multidot(n, 0, W.V, bvec, W.partial, hd, st));
  AH_HIP(hipMemcpyAsync(hh, hd, sizeof(double), hipMemcpyDeviceToHost, st));
  AH_HIP(hipStreamSynchronize(st));
  const double bnorm = std::sqrt(hh[0]);
  if (!(bnorm > 0.0)) {
    AH_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
    if (info) { info->iters = 0; info->converged = 1; info->relres = 0; info->true_relres = 0; }
    return AH_OK;
  }
  if (!std::isfinite(bnorm)) { set_error("air_solve: non-finite right-hand side"); return AH_EBREAKDOWN; }
  // Hr: Hessenberg columns as formed (rows 0..m); Hg: the same after the
  // Givens rotations; Rt: the triangular factor of Z~ = Z R
  std::vector<double> Hr((size_t)(m + 1) * m), Hg((size_t)(m + 1) * m), Rt((size_t)m * m), cs(m), sn(m),
      g(m + 1), y(m), t(m);
  int its = 0;
  bool converged = false;
  double relres = 1.0, true_rel = 1.0;
  ah_status status = AH_OK;
  while (true) {
    // u_0 = r = b - A x, the first candidate (r_00 = ||r||)
    AH_TRY((op_apply<double, SP_RES>(A, G0, n, x, bvec, W.V, st)));
    AH_TRY(multidot(n, 0, W.V, W.V, W.partial, hd, st));
    AH_HIP(hipMemcpyAsync(hh, hd, sizeof(double), hipMemcpyDeviceToHost, st));
    AH_HIP(hipStreamSynchronize(st));
    const double beta = std::sqrt(hh[0]);
    true_rel = beta / bnorm;
    relres = true_rel;
    if (!std::isfinite(beta)) { set_error("air_solve: breakdown (NaN residual)"); status = AH_EBREAKDOWN; break; }
    if (beta <= prm.tol * bnorm) { converged = true; break; }
    if (its >= prm.maxit) break;
    std::fill(Hr.begin(), Hr.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int kdone = 0;
    double wnorm_prev = 0.0;   // ||A z_{j-1}||, for the breakdown test
    for (int j = 0; j <= m; ++j) {
      double* uj = W.V + (int64_t)j * n;
      const bool more = j < m && its + (j >= 1 ? 1 : 0) < prm.maxit;
      if (more) {
        double* zj = W.Z ? W.Z + (int64_t)j * n : nullptr;
        float* zj32 = W.Z32 ? W.Z32 + (int64_t)j * n : nullptr;
        AH_TRY(precond(h, uj, prm.precision == 0 ? zj : nullptr, prm.precision == 1 ? zj32 : nullptr,
                       prm.precision, transpose, st));
        const double by = op_mv_bytes(h, A, n, prm.precision ? 4.0 : 8.0);
        if (prm.precision == 0)
          AH_TRY((op_apply<double, SP_MV>(A, G0, n, zj, (const double*)nullptr, W.w, st,
                                          transpose ? nullptr : "spmv0", by)));
        else
          AH_TRY((op_apply<float, SP_MV>(A, G0, n, zj32, (const double*)nullptr, W.w, st,
                                         transpose ? nullptr : "spmv0", by)));
      }
      {
        ProfScope ps;
        prof_begin(ps, transpose ? nullptr : "arnoldi_dot", st, (double)(j + 2) * n * 8.0);
        hipLaunchKernelGGL(k_dcgs_dot, dim3(nblk, (unsigned)std::max<int64_t>(1, cdiv(j, DD_V))), dim3(256), 0, st,
                           n, j, W.V, more ? W.w : nullptr, W.partial, nblk);
        prof_end(ps);
        AH_LAUNCHED();
      }
      hipLaunchKernelGGL(k_reduce_partial, dim3(2 * j + 3), dim3(256), 0, st, nblk, W.partial, hd, 0);
      AH_LAUNCHED();
      AH_HIP(hipMemcpyAsync(hh, hd, (2 * j + 3) * sizeof(double), hipMemcpyDeviceToHost, st));
      AH_HIP(hipStreamSynchronize(st));
      const double* a = hh;
      const double* c = hh + j;
      const double alpha = hh[2 * j], gamma = hh[2 * j + 1], omega = hh[2 * j + 2];
      double aa = 0.0, ac = 0.0;
      for (int i = 0; i < j; ++i) { aa += a[i] * a[i]; ac += a[i] * c[i]; }
      if (!std::isfinite(alpha) || !std::isfinite(gamma) || !std::isfinite(omega) || !std::isfinite(aa)) {
        set_error("air_solve: breakdown (NaN in Arnoldi)");
        status = AH_EBREAKDOWN;
        break;
      }
      const double rjj = alpha > aa ? std::sqrt(alpha - aa) : 0.0;
      if (j >= 1) {
        // column j-1 is complete: A z_{j-1} = Q (h + a) + r_jj q_j
        const int k = j - 1;
        for (int i = 0; i < j; ++i) Hr[(size_t)i * m + k] += a[i];
        Hr[(size_t)j * m + k] = rjj;
        for (int i = 0; i <= j; ++i) Hg[(size_t)i * m + k] = Hr[(size_t)i * m + k];
        for (int i = 0; i < k; ++i) {
          const double p = Hg[(size_t)i * m + k], q = Hg[(size_t)(i + 1) * m + k];
          Hg[(size_t)i * m + k] = cs[i] * p + sn[i] * q;
          Hg[(size_t)(i + 1) * m + k] = -sn[i] * p + cs[i] * q;
        }
        const double p = Hg[(size_t)k * m + k], q = Hg[(size_t)j * m + k];
        const double den = std::hypot(p, q);
        if (den == 0.0) { cs[k] = 1.0; sn[k] = 0.0; } else { cs[k] = p / den; sn[k] = q / den; }
        Hg[(size_t)k * m + k] = cs[k] * p + sn[k] * q;
        Hg[(size_t)j * m + k] = 0.0;
        g[j] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        ++its;
        kdone = j;
        relres = std::fabs(g[j]) / bnorm;
        const bool happy = rjj <= 1e-14 * wnorm_prev;
        if (std::fabs(g[j]) <= prm.tol * bnorm || happy || its >= prm.maxit) break;
      }
      if (!more || !(rjj > 0.0)) break;
      // R column j, then Hessenberg column j as formed (rows 0..j)
      for (int i = 0; i < j; ++i) Rt[(size_t)i * m + j] = a[i];
      Rt[(size_t)j * m + j] = rjj;
      const double d = (gamma - ac) / rjj;
      for (int i = 0; i <= j; ++i) {
        double s = i < j ? c[i] : d;
        for (int l = std::max(0, i - 1); l < j; ++l) s -= Hr[(size_t)i * m + l] * a[l];
        Hr[(size_t)i * m + j] = s / rjj;
      }
      wnorm_prev = std::sqrt(omega) / rjj;
      for (int i = 0; i < j; ++i) { coef_h[i] = a[i]; coef_h[j + i] = c[i]; }
      coef_h[2 * j] = d;
      coef_h[2 * j + 1] = 1.0 / rjj;
      AH_HIP(hipMemcpyAsync(coef_d, coef_h, (2 * j + 2) * sizeof(double), hipMemcpyHostToDevice, st));
      {
        ProfScope ps;
        prof_begin(ps, transpose ? nullptr : "arnoldi_update", st, (double)(j + 4) * n * 8.0);
        hipLaunchKernelGGL(k_dcgs_update, dim3(nblk), dim3(256), (unsigned)((2 * j + 2) * sizeof(double)), st, n, j,
                           W.V, W.w, coef_d);
        prof_end(ps);
        AH_LAUNCHED();
      }
    }
    if (status != AH_OK && kdone == 0) break;
    // y from the rotated Hessenberg, then t = R^-1 y, x += Z~ t
    for (int i = kdone - 1; i >= 0; --i) {
      double s = g[i];
      for (int cc = i + 1; cc < kdone; ++cc) s -= Hg[(size_t)i * m + cc] * y[cc];
      y[i] = s / Hg[(size_t)i * m + i];
    }
    for (int i = kdone - 1; i >= 0; --i) {
      double s = y[i];
      for (int cc = i + 1; cc < kdone; ++cc) s -= Rt[(size_t)i * m + cc] * t[cc];
      t[i] = s / Rt[(size_t)i * m + i];
    }
    for (int i = 0; i < kdone; ++i) coef_h[i] = t[i];
    AH_HIP(hipMemcpyAsync(coef_d, coef_h, kdone * sizeof(double), hipMemcpyHostToDevice, st));
    if (kdone > 0) {
      if (prm.precision == 0)
        hipLaunchKernelGGL(k_maxpy<double>, g1(n), dim3(256), 0, st, n, kdone, W.Z, n, coef_d, x, 1.0);
      else
        hipLaunchKernelGGL(k_maxpy<float>, g1(n), dim3(256), 0, st, n, kdone, W.Z32, n, coef_d, x, 1.0);
      AH_LAUNCHED();
    }
    if (status != AH_OK) break;
  }
  AH_HIP(hipStreamSynchronize(st));
  if (info) {
    info->iters = its;
    info->converged = converged ? 1 : 0;
    info->relres = relres;
    info->true_relres = true_rel;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status != AH_OK) return status;
  return converged ? AH_OK : AH_ENOCONV;
}

// Right-preconditioned BiCGSTAB (the paper's Krylov method, Section 4) on
// A x = b: per step p_hat = M p, v = A p_hat, s = r - alpha v, then
// s_hat = M s, t = A s_hat, x += alpha p_hat + omega s_hat, r = s - omega t.
// The scalars stay on the device; the host reads ||s|| and ||r|| once per
// half step.  Convergence is confirmed by the true residual; a vanishing
// or non-finite rho, r_hat.v or omega restarts from the current iterate.
static ah_status bicgstab(ah_hier* h, Op A, const double* bvec, double* x, const ah_solve_params& prm,
                          int transpose, hipStream_t st, ah_solve_info* info) {
  const int64_t n = h->lev[0].n;
  // workspace: 8 vectors, then 3072 reduction partials (two dots of at most
  // 1024 blocks each), then the BC_N device scalars
  if (!h->bcg) {
    h->arena.stream = st;
    AH_TRY(h->arena.get(&h->bcg, 8 * n + 3072 + 16));
  }
  if (prm.precision == 1 && !h->bcg32) {
    h->arena.stream = st;
    AH_TRY(h->arena.get(&h->bcg32, n));
  }
  double* r = h->bcg;
  double* rh = r + n;
  double* p = rh + n;
  double* v = p + n;
  double* sv = v + n;
  double* tv = sv + n;
  double* ph = tv + n;
  double* sh = ph + n;
  double* part = h->bcg + 8 * n;
  double* sc = part + 3072;
  const int G0 = op_lanes(h, A, n);
  const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(n, 256 * 4)));
  double* hh = pinned_scratch(16);
  if (!hh) { set_error("pinned host allocation failed"); return AH_ENOMEM; }
  auto read_sc = [&](int count) -> ah_status {
    AH_HIP(hipMemcpyAsync(hh, sc, count * sizeof(double), hipMemcpyDeviceToHost, st));
    AH_HIP(hipStreamSynchronize(st));
    return AH_OK;
  };
  auto apply_m = [&](const double* in, double* out) -> ah_status {
    if (prm.precision == 0) return precond(h, in, out, nullptr, 0, transpose, st);
    AH_TRY(precond(h, in, nullptr, h->bcg32, 1, transpose, st));
    hipLaunchKernelGGL((k_cast<float, double>), g1(n), dim3(256), 0, st, n, h->bcg32, out);
    AH_LAUNCHED();
    return AH_OK;
  };
  auto spmv = [&](const double* in, double* out) -> ah_status {
    return op_apply<double, SP_MV>(A, G0, n, in, (const double*)nullptr, out, st, transpose ? nullptr : "spmv0",
                                   op_mv_bytes(h, A, n, 8.0));
  };
  auto t0 = std::chrono::steady_clock::now();
  AH_TRY(multidot(n, 0, rh, bvec, part, sc, st));
  AH_TRY(read_sc(1));
  const double bnorm = std::sqrt(hh[0]);
  int its = 0;
  bool converged = false;
  double relres = 1.0, true_rel = 1.0;
  ah_status status = AH_OK;
  if (!(bnorm > 0.0)) {
    AH_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
    if (info) { info->iters = 0; info->converged = 1; info->relres = 0; info->true_relres = 0; }
    return AH_OK;
  }
  if (!std::isfinite(bnorm)) { set_error("air_solve: non-finite right-hand side"); return AH_EBREAKDOWN; }
  const double ones[3] = {1.0, 1.0, 1.0};
  while (true) {
    // (re)start: r = b - A x, r_hat = r, p = v = 0, rho_old = alpha = omega = 1
    AH_TRY((op_apply<double, SP_RES>(A, G0, n, x, bvec, r, st)));
    AH_TRY(multidot(n, 0, rh, r, part, sc + BC_RR, st));
    AH_TRY(read_sc(BC_N));
    true_rel = std::sqrt(hh[BC_RR]) / bnorm;
    relres = true_rel;
    if (!std::isfinite(true_rel)) { set_error("air_solve: breakdown (NaN residual)"); status = AH_EBREAKDOWN; break; }
    if (true_rel <= prm.tol) { converged = true; break; }
    if (its >= prm.maxit) break;
    AH_HIP(hipMemcpyAsync(rh, r, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    AH_HIP(hipMemsetAsync(p, 0, 2 * n * sizeof(double), st));   // p and v
    std::memcpy(hh + 8, ones, sizeof(ones));
    AH_HIP(hipMemcpyAsync(sc + BC_RHOOLD, hh + 8, 3 * sizeof(double), hipMemcpyHostToDevice, st));
    bool restart = false;
    while (its < prm.maxit) {
      AH_TRY(multidot(n, 1, rh, r, part, sc + BC_RHO, st));      // rho, r.r
      hipLaunchKernelGGL(k_bicg_p, g1(n), dim3(256), 0, st, n, r, v, p, sc);
      AH_LAUNCHED();
      AH_TRY(apply_m(p, ph));
      AH_TRY(spmv(ph, v));
      ++its;
      AH_TRY(multidot(n, 1, rh, v, part, sc + BC_RV, st));      // r_hat.v, v.v
      hipLaunchKernelGGL(k_bicg_s, dim3(nblk), dim3(256), 0, st, n, r, v, sv, sc, part, nblk);
      AH_LAUNCHED();
      hipLaunchKernelGGL(k_reduce_partial, dim3(1), dim3(256), 0, st, nblk, part, sc + BC_SS, 0);
      AH_LAUNCHED();
      AH_TRY(read_sc(BC_N));
      const double snorm = std::sqrt(hh[BC_SS]);
      if (!std::isfinite(snorm) || hh[BC_RHO] == 0.0 || hh[BC_RV] == 0.0) { restart = true; break; }
      if (snorm <= prm.tol * bnorm) {
        hipLaunchKernelGGL(k_bicg_xhalf, g1(n), dim3(256), 0, st, n, ph, x, sc);
        AH_LAUNCHED();
        relres = snorm / bnorm;
        break;
      }
      AH_TRY(apply_m(sv, sh));
      AH_TRY(spmv(sh, tv));
      AH_TRY(multidot(n, 1, sv, tv, part, sc + BC_ST, st));     // s.t, t.t
      hipLaunchKernelGGL(k_bicg_xr, dim3(nblk), dim3(256), 0, st, n, ph, sh, sv, tv, x, r, sc, part, nblk);
      AH_LAUNCHED();
      hipLaunchKernelGGL(k_reduce_partial, dim3(1), dim3(256), 0, st, nblk, part, sc + BC_RR, 0);
      AH_LAUNCHED();
      AH_TRY(read_sc(BC_N));
      const double rnorm = std::sqrt(hh[BC_RR]);
      relres = rnorm / bnorm;
      if (!std::isfinite(rnorm)) { restart = true; break; }
      if (rnorm <= prm.tol * bnorm || hh[BC_OMEGA] == 0.0) break;
    }
    (void)restart;   // either way the outer loop recomputes the true residual
  }
  AH_HIP(hipStreamSynchronize(st));
  if (info) {
    info->iters = its;
    info->converged = converged ? 1 : 0;
    info->relres = relres;
    info->true_relres = true_rel;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status != AH_OK) return status;
  return converged ? AH_OK : AH_ENOCONV;
}

// ------------------------------------------------ allocation-free solve
// The FGMRES workspace of air_solve_noalloc lives in this file-scope device
// array (one copy per GPU, held until the process ends).  In host code the
// name is only a stand-in for the symbol: the device address of each GPU's
// copy comes from hipGetSymbolAddress, looked up once per device with that
// device current, and only that address is passed to kernels.
constexpr size_t kScratchBytes = (size_t)AH_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<char*> g_scratch_addr;   // indexed by device id

static ah_status scratch_address(char** out) {
  int dev = 0;
  AH_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("air_solve_noalloc: hipGetSymbolAddress of the scratch array failed (%s)", hipGetErrorString(e));
      return AH_EHIP;
    }
    g_scratch_addr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_addr[dev];
  return AH_OK;
}

// Lays the FGMRES workspace for n unknowns and restart m out from base in
// 256-byte aligned pieces (base == nullptr: sizes only); returns the bytes.
static size_t carve_workspace(char* base, int64_t n, int m, int precision, KWork* W) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const size_t nd = (size_t)n * sizeof(double);
  W->V = reinterpret_cast<double*>(take((size_t)(m + 1) * nd));
  if (precision == 0)
    W->Z = reinterpret_cast<double*>(take((size_t)m * nd));
  else
    W->Z32 = reinterpret_cast<float*>(take((size_t)m * (size_t)n * sizeof(float)));
  W->w = reinterpret_cast<double*>(take(nd));
  W->r = reinterpret_cast<double*>(take(nd));
  W->bhat = reinterpret_cast<double*>(take(nd));
  W->partial = reinterpret_cast<double*>(take((size_t)(2 * m + 4) * 1024 * sizeof(double)));
  W->hdev = reinterpret_cast<double*>(take((size_t)4 * (m + 3) * sizeof(double)));
  return off;
}

}  // namespace ah

using namespace ah;

extern "C" void ah_solve_defaults(ah_solve_params* p) {
  if (!p) return;
  p->tol = 1e-8;
  p->restart = 100;
  p->maxit = 1000;
  p->precision = 0;
  p->x0_given = 0;
  p->method = 0;
}

static ah_status check_solve(const ah_hier* h, const ah_solve_params* prm, int transpose) {
  if (!h || !prm) { set_error("air_solve: null argument"); return AH_EINVAL; }
  if (prm->precision == 1 && !h->prm.fp32_cycle) {
    set_error("air_solve: FP32 cycle requested but the hierarchy was built without fp32_cycle");
    return AH_EINVAL;
  }
  if (prm->precision < 0 || prm->precision > 1 || prm->restart < 1 || prm->maxit < 0 || !(prm->tol > 0.0) ||
      prm->method < 0 || prm->method > 1) {
    set_error("air_solve: invalid parameters");
    return AH_EINVAL;
  }
  if (transpose && !h->prm.adjoint) {
    set_error("air_solve_adjoint: hierarchy built without adjoint = 1");
    return AH_EINVAL;
  }
  return AH_OK;
}

// Forward solve with a given workspace (W.bhat holds the scaled
// right-hand side when rhs is given).
static ah_status solve_forward(ah_hier* h, const KWork& W, const double* rhs, double* x, const ah_solve_params& prm,
                               hipStream_t st, ah_solve_info* info) {
  const ah_system* s = h->sys;
  const int64_t n = s->n;
  const double* b = s->d_Hhat;
  if (rhs) {
    hipLaunchKernelGGL(k_blockscale, g1(n), dim3(256), 0, st, s->nfree, s->b, s->d_Dinv, rhs, W.bhat, 0);
    AH_LAUNCHED();
    b = W.bhat;
  }
  if (!prm.x0_given) AH_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
  Op A{s->d_rowptr, s->d_col, s->d_val};
  const AhLevel& L0 = h->lev[0];
  if (L0.ob) {
    A.ob = L0.ob;
    A.optr = L0.optr;
    A.ocol = L0.ocol;
    A.ov = L0.oval;
    A.nov = L0.nov;
    A.lpb = h->fbb ? (h->lpb ? h->lpb : fbb_lanes(L0.nov, n, L0.ob)) : 0;
  }
  if (prm.method == 1) return bicgstab(h, A, b, x, prm, 0, st, info);
  return fgmres(h, W, A, b, x, prm, 0, st, info);
}

extern "C" ah_status air_solve(const ah_hier* hc, const double* rhs, double* x, const ah_solve_params* prm,
                               void* stream, ah_solve_info* info) {
  AH_TRY(check_solve(hc, prm, 0));
  if (hc->sys->n == 0) {   // nothing to solve
    if (info) { std::memset(info, 0, sizeof(*info)); info->converged = 1; }
    return AH_OK;
  }
  if (!x) { set_error("air_solve: null x"); return AH_EINVAL; }
  ah_hier* h = const_cast<ah_hier*>(hc);
  hipStream_t st = as_stream(stream);
  KWork W;
  AH_TRY(ensure_workspace(h, std::max(1, prm->restart), prm->precision, st, &W));
  return solve_forward(h, W, rhs, x, *prm, st, info);
}

extern "C" ah_status air_solve_noalloc(const ah_hier* hc, const double* rhs, double* x,
                                       const ah_solve_params* prm, void* stream, ah_solve_info* info) {
  AH_TRY(check_solve(hc, prm, 0));
  if (prm->method != 0) {
    set_error("air_solve_noalloc: only FGMRES (method 0) runs without allocation");
    return AH_EUNSUPPORTED;
  }
  if (prm->restart > AH_NOALLOC_MAX_RESTART) {
    set_error("air_solve_noalloc: restart %d exceeds %d", prm->restart, AH_NOALLOC_MAX_RESTART);
    return AH_EUNSUPPORTED;
  }
  if (hc->sys->n == 0) {
    if (info) { std::memset(info, 0, sizeof(*info)); info->converged = 1; }
    return AH_OK;
  }
  if (!x) { set_error("air_solve_noalloc: null x"); return AH_EINVAL; }
  ah_hier* h = const_cast<ah_hier*>(hc);
  hipStream_t st = as_stream(stream);
  const int m = std::max(1, prm->restart);
  const int64_t n = h->sys->n;
  KWork W;
  const size_t need = carve_workspace(nullptr, n, m, prm->precision, &W);
  if (need > kScratchBytes) {
    set_error("air_solve_noalloc: workspace of %zu bytes (n = %lld, restart = %d) exceeds the %zu-byte scratch array",
              need, (long long)n, m, kScratchBytes);
    return AH_EUNSUPPORTED;
  }
  char* base = nullptr;
  AH_TRY(scratch_address(&base));
  carve_workspace(base, n, m, prm->precision, &W);
  static thread_local double stage[4 * (AH_NOALLOC_MAX_RESTART + 3)];   // pageable host staging
  W.host = stage;
  return solve_forward(h, W, rhs, x, *prm, st, info);
}

extern "C" ah_status air_solve_adjoint(const ah_hier* hc, const double* g, double* lam, const ah_solve_params* prm,
                                       void* stream, ah_solve_info* info) {
  AH_TRY(check_solve(hc, prm, 1));
  if (hc->sys->n == 0) {
    if (info) { std::memset(info, 0, sizeof(*info)); info->converged = 1; }
    return AH_OK;
  }
  if (!g || !lam) { set_error("air_solve_adjoint: null argument"); return AH_EINVAL; }
  ah_hier* h = const_cast<ah_hier*>(hc);
  hipStream_t st = as_stream(stream);
  const ah_system* s = h->sys;
  const int64_t n = s->n;
  KWork W;
  AH_TRY(ensure_workspace(h, std::max(1, prm->restart), prm->precision, st, &W));
  double* mu = W.bhat;   // S_hat^T mu = g, then lam = D_b^-T mu
  AhLevel& L0 = h->lev[0];
  if (!L0.ATptr && !L0.otval) {
    set_error("air_solve_adjoint: transposed level-0 operator missing");
    return AH_EINVAL;
  }
  AH_HIP(hipMemsetAsync(mu, 0, n * sizeof(double), st));   // zero initial guess
  Op AT{L0.ATptr, L0.ATcol, L0.ATval};
  if (L0.otval) {
    AT.ob = L0.ob;
    AT.optr = L0.optr;
    AT.ocol = L0.ocol;
    AT.ov = L0.otval;
    AT.nov = L0.nov;
    AT.lpb = h->fbb ? (h->lpb ? h->lpb : fbb_lanes(L0.nov, n, L0.ob)) : 0;
  }
  ah_status rc = prm->method == 1 ? bicgstab(h, AT, g, mu, *prm, 1, st, info)
                                   : fgmres(h, W, AT, g, mu, *prm, 1, st, info);
  if (rc < 0) return rc;
  hipLaunchKernelGGL(k_blockscale, g1(n), dim3(256), 0, st, s->nfree, s->b, s->d_Dinv, mu, lam, 1);
  AH_LAUNCHED();
  AH_HIP(hipStreamSynchronize(st));
  return rc;
}

extern "C" ah_status ah_vcycle_apply(const ah_hier* hc, const double* r, double* z, int precision, int transpose,
                                     void* stream) {
  if (!hc || !r || !z) { set_error("ah_vcycle_apply: null argument"); return AH_EINVAL; }
  ah_hier* h = const_cast<ah_hier*>(hc);
  if (precision == 1 && !h->prm.fp32_cycle) { set_error("ah_vcycle_apply: no FP32 operators"); return AH_EINVAL; }
  if (transpose && !h->prm.adjoint) { set_error("ah_vcycle_apply: no transposes"); return AH_EINVAL; }
  hipStream_t st = as_stream(stream);
  const int64_t n = h->lev[0].n;
  if (precision == 0) return precond(h, r, z, nullptr, 0, transpose, st);
  float* z32 = nullptr;
  Arena tmp;
  tmp.stream = st;
  AH_TRY(tmp.get(&z32, n));
  AH_TRY(precond(h, r, nullptr, z32, 1, transpose, st));
  hipLaunchKernelGGL((k_cast<float, double>), g1(n), dim3(256), 0, st, n, z32, z);
  AH_LAUNCHED();
  AH_HIP(hipStreamSynchronize(st));
  tmp.release();
  return AH_OK;
}
