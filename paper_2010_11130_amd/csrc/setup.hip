// air_setup: lAIR algebraic multigrid hierarchy on the scaled facet system
// treated as a scalar matrix (Section 3; solver settings of Section 4).
//
// Per level: strength of connection (row-wise |a_ij| >= theta max_{k!=i}
// |a_ik| (1-1e-12)), PMIS C/F splitting with integer keys
// (influence count << 44 | 44-bit bijective hash of the index), one-point
// interpolation (strongest strong C neighbour, ties to the smallest index),
// distance-one lAIR restriction rows from local dense solves
// A[N_i,N_i]^T z = -A[i,N_i]^T (one wave per C point, LU with partial
// pivoting in LDS), and the Galerkin product A_c = R A P (one wave per
// coarse row, LDS hash; P is one-point so A P is a column relabelling).
// The coarsest matrix is inverted densely in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include <queue>

#include "prof.h"
#include "system.h"

namespace ah {

__device__ inline uint64_t hash44(uint64_t i, int level) {
  const uint64_t M = (1ull << 44) - 1;
  uint64_t x = (i + (((uint64_t)(level + 1) * 0x9E3779B97F4A7C15ull) & M)) & M;
  x ^= x >> 21;
  x = (x * (0xBF58476D1CE4E5B9ull & M)) & M;
  x ^= x >> 19;
  x = (x * (0x94D049BB133111EBull & M)) & M;
  x ^= x >> 22;
  return x;
}

// Strength of connection, 16 lanes per row: row max of the off-diagonal
// magnitudes by a cross-lane reduction, then the marks.
constexpr int SG = 16;
__global__ __launch_bounds__(256) void k_strength(int64_t n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                  double theta, uint8_t* __restrict__ strong,
                                                  int32_t* __restrict__ infl) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gid / SG;
  const int g = (int)(gid % SG);
  if (i >= n) return;
  const int64_t k0 = rp[i], k1 = rp[i + 1];
  double m = 0.0;
  for (int64_t k = k0 + g; k < k1; k += SG)
    if (ci[k] != i) m = fmax(m, fabs(v[k]));
  for (int o = SG / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, SG));
  const double thr = theta * m * (1.0 - 1e-12);
  for (int64_t k = k0 + g; k < k1; k += SG) {
    bool sflag = ci[k] != i && m > 0.0 && fabs(v[k]) >= thr;
    strong[k] = sflag;
    if (sflag) atomicAdd(&infl[ci[k]], 1);
  }
}

// state: 0 undecided, 1 C, 2 F
__global__ void k_pmis_init(int64_t n, const int32_t* __restrict__ infl, int level, uint64_t* __restrict__ key,
                            int8_t* __restrict__ state) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = ((uint64_t)infl[i] << 44) | hash44((uint64_t)i, level);
  state[i] = infl[i] == 0 ? 2 : 0;
}

// 8 lanes per row for the PMIS phases and the one-point kernel.
constexpr int PG = 8;

// The round kernels visit rows 0 .. n-1, or the rows list[0 .. n-1] (the
// points still undecided when the list was made; points only leave that
// state, so the rows outside the list are no-ops of the round); with nd,
// the list's length is *nd (at most n, the bound the grid was sized for).
__global__ __launch_bounds__(256) void k_pmis_nbmax(int64_t n, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const uint8_t* __restrict__ strong,
                                                    const uint64_t* __restrict__ key, const int8_t* __restrict__ state,
                                                    unsigned long long* __restrict__ nbmax,
                                                    const int32_t* __restrict__ list, const int64_t* __restrict__ nd) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ii = gid / PG;
  const int g = (int)(gid % PG);
  if (nd) n = *nd;
  if (ii >= n) return;
  const int64_t i = list ? (int64_t)list[ii] : ii;
  if (state[i] != 0) return;
  unsigned long long mx = 0, ki = key[i];
  for (int64_t k = rp[i] + g; k < rp[i + 1]; k += PG) {
    // the flag and the column together (no branch between the two loads)
    const bool sk = strong[k] != 0;
    const int32_t j = ci[k];
    if (!sk) continue;
    if (state[j] != 0) continue;
    mx = mx > key[j] ? mx : key[j];
    atomicMax(&nbmax[j], ki);      // i depends on j: i is a neighbour of j as well
  }
  for (int o = PG / 2; o > 0; o >>= 1) {
    unsigned long long other = __shfl_xor(mx, o, PG);
    mx = mx > other ? mx : other;
  }
  if (g == 0 && mx) atomicMax(&nbmax[i], mx);
}

// New C points: undecided points whose key beats every undecided neighbour.
// nbmax is reset for the next round (only undecided points carry a value),
// and the round's undecided flag is cleared.
__global__ void k_pmis_select(int64_t n, const uint64_t* __restrict__ key, unsigned long long* __restrict__ nbmax,
                              int8_t* __restrict__ state, unsigned long long* __restrict__ left,
                              const int32_t* __restrict__ list, const int64_t* __restrict__ nd) {
  const int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ii == 0) *left = 0;
  if (nd) n = *nd;
  if (ii >= n) return;
  const int64_t i = list ? (int64_t)list[ii] : ii;
  if (state[i] != 0) return;
  if (key[i] > nbmax[i]) state[i] = 1;
  nbmax[i] = 0;
}

// Undecided points with a strong C neighbour become F. The kernels with a
// per-launch result use a capped grid (grid-stride over rows) and one
// global write per block: a write per wave to one address serializes.
__global__ __launch_bounds__(256) void k_pmis_fmark(int64_t n, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const uint8_t* __restrict__ strong, int8_t* __restrict__ state,
                                                    unsigned long long* __restrict__ left,
                                                    const int32_t* __restrict__ list,
                                                    const int64_t* __restrict__ nd) {
  const int g = (int)(threadIdx.x % PG);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / PG);
  int undecided = 0;
  if (nd) n = *nd;
  for (int64_t ii = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PG; ii < n; ii += stride) {
    const int64_t i = list ? (int64_t)list[ii] : ii;
    if (state[i] != 0) continue;
    int hit = 0;
    for (int64_t k = rp[i] + g; k < rp[i + 1]; k += PG)
      if (strong[k] && state[ci[k]] == 1) hit = 1;
    for (int o = PG / 2; o > 0; o >>= 1) hit |= __shfl_xor(hit, o, PG);
    if (!hit) undecided = 1;
    else if (g == 0) state[i] = 2;
  }
  if (__syncthreads_or(undecided) && threadIdx.x == 0) *left = 1ull;
}

// Every PMIS round of a small level in one workgroup: keys, neighbour maxima
// and states live in LDS (17 bytes per row), the strength graph is read from
// global memory, phases are separated by barriers.  Same rounds as
// k_pmis_nbmax / k_pmis_select / k_pmis_fmark, so the same splitting.
// Dynamic LDS: n (8 + 8 + 1) bytes (8-byte aligned).  *err is set if the
// rounds exceed n + 1 (cannot happen: the largest undecided key always
// becomes C).
constexpr int PMIS_WG_MAX = 8192;

__global__ __launch_bounds__(1024) void k_pmis_wg(int n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  const uint8_t* __restrict__ strong,
                                                  const uint64_t* __restrict__ key_g, int8_t* __restrict__ state_g,
                                                  unsigned long long* __restrict__ err) {
  extern __shared__ __align__(16) unsigned long long pm[];
  unsigned long long* key = pm;
  unsigned long long* nb = pm + n;
  int8_t* st = reinterpret_cast<int8_t*>(pm + 2 * n);
  const int t = threadIdx.x, NT = blockDim.x;
  for (int i = t; i < n; i += NT) {
    key[i] = key_g[i];
    nb[i] = 0ull;
    st[i] = state_g[i];
  }
  __syncthreads();
  for (int round = 0;; ++round) {
    if (round > n + 1) {
      if (t == 0) atomicOr(err, 1ull);
      break;
    }
    // largest undecided key among the symmetrised strong neighbours
    for (int i = t; i < n; i += NT) {
      if (st[i] != 0) continue;
      unsigned long long mx = 0ull;
      const unsigned long long ki = key[i];
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (!strong[k]) continue;
        const int32_t j = ci[k];
        if (st[j] != 0) continue;
        mx = mx > key[j] ? mx : key[j];
        atomicMax(&nb[j], ki);
      }
      if (mx) atomicMax(&nb[i], mx);
    }
    __syncthreads();
    for (int i = t; i < n; i += NT) {
      if (st[i] != 0) continue;
      if (key[i] > nb[i]) st[i] = 1;
      nb[i] = 0ull;
    }
    __syncthreads();
    int undecided = 0;
    for (int i = t; i < n; i += NT) {
      if (st[i] != 0) continue;
      int hit = 0;
      for (int64_t k = rp[i]; k < rp[i + 1] && !hit; ++k)
        if (strong[k] && st[ci[k]] == 1) hit = 1;
      if (hit) st[i] = 2;
      else undecided = 1;
    }
    if (!__syncthreads_or(undecided)) break;
  }
  for (int i = t; i < n; i += NT) state_g[i] = st[i];
}

__global__ void k_cf_flags(int64_t n, const int8_t* __restrict__ state, int8_t* __restrict__ cf,
                           int32_t* __restrict__ isc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int8_t c = state[i] == 1;
  cf[i] = c;
  isc[i] = c;
}

// One-point interpolation; for C points the lAIR row length 1 + |N_i| and
// the number of R A P candidates of its coarse row (row lengths of A over
// {i} and N_i); for F points their list and the F-row statistics (count,
// entries).
// imax[0] = max |N_i|, imax[1] = max candidates, imax[2] = max length of a
// C row; fst[0..1] = F rows, entries.
// PG lanes per row; the strongest C neighbour is the first in row order
// (smallest column) within relative 1e-12 of the maximum.  fsearch = 0
// (block AIR, whose P comes from the block graph): F rows only listed.
__global__ __launch_bounds__(256) void k_onepoint(int64_t n, int fsearch, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                  const uint8_t* __restrict__ strong,
                                                  const uint8_t* __restrict__ strong_r, const int8_t* __restrict__ cf,
                                                  const int64_t* __restrict__ cidx, int32_t* __restrict__ pcol,
                                                  int32_t* __restrict__ rcnt, int32_t* __restrict__ clist,
                                                  int32_t* __restrict__ flist, int* __restrict__ imax,
                                                  unsigned long long* __restrict__ fst) {
  const int g = (int)(threadIdx.x % PG);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / PG);
  int mmax = 0, cmax = 0, omax = 0;
  unsigned long long fcnt = 0, fent = 0;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PG; i < n; i += stride) {
    const int64_t k0 = rp[i], k1 = rp[i + 1];
    if (cf[i]) {
      int m = 0;
      int64_t cand = 0;
      for (int64_t k = k0 + g; k < k1; k += PG) {
        const bool sk = strong_r[k] != 0;
        const int32_t c = ci[k];
        if (sk && !cf[c]) {
          ++m;
          cand += rp[c + 1] - rp[c];
        }
      }
      for (int o = PG / 2; o > 0; o >>= 1) {
        m += __shfl_xor(m, o, PG);
        cand += __shfl_xor(cand, o, PG);
      }
      if (g == 0) {
        cand += k1 - k0;
        pcol[i] = (int32_t)cidx[i];
        rcnt[cidx[i]] = 1 + m;
        clist[cidx[i]] = (int32_t)i;
        mmax = m > mmax ? m : mmax;
        omax = (int)(k1 - k0) > omax ? (int)(k1 - k0) : omax;
        const int c = cand > 0x3fffffff ? 0x3fffffff : (int)cand;
        cmax = c > cmax ? c : cmax;
      }
      continue;
    }
    double mx = -1.0;
    if (fsearch)
      for (int64_t k = k0 + g; k < k1; k += PG) {
        const bool sk = strong[k] != 0;
        const int32_t c = ci[k];
        const double a = fabs(v[k]);
        if (sk && cf[c]) mx = fmax(mx, a);
      }
    for (int o = PG / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, PG));
    int64_t first = k1;
    if (mx >= 0.0) {
      const double thr = mx * (1.0 - 1e-12);
      for (int64_t k = k0 + g; k < k1; k += PG) {
        const bool sk = strong[k] != 0;
        const int32_t c = ci[k];
        const double a = fabs(v[k]);
        if (sk && cf[c] && a >= thr) { first = k; break; }
      }
      for (int o = PG / 2; o > 0; o >>= 1) {
        int64_t other = __shfl_xor(first, o, PG);
        first = other < first ? other : first;
      }
    }
    if (g == 0) {
      if (fsearch) pcol[i] = first < k1 ? (int32_t)cidx[ci[first]] : -1;
      flist[i - cidx[i]] = (int32_t)i;   // F points in increasing order
      fcnt += 1;
      fent += (unsigned long long)(k1 - k0);
    }
  }
  // block totals, one atomic each
  for (int o = 32; o > 0; o >>= 1) {
    int a = __shfl_xor(mmax, o, 64), c = __shfl_xor(cmax, o, 64), ow = __shfl_xor(omax, o, 64);
    mmax = a > mmax ? a : mmax;
    cmax = c > cmax ? c : cmax;
    omax = ow > omax ? ow : omax;
    fcnt += __shfl_xor(fcnt, o, 64);
    fent += __shfl_xor(fent, o, 64);
  }
  __shared__ int sm[3][4];
  __shared__ unsigned long long su[2][4];
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    sm[0][w] = mmax; sm[1][w] = cmax; sm[2][w] = omax;
    su[0][w] = fcnt; su[1][w] = fent;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x / 64); ++k) {
      mmax = sm[0][k] > mmax ? sm[0][k] : mmax;
      cmax = sm[1][k] > cmax ? sm[1][k] : cmax;
      omax = sm[2][k] > omax ? sm[2][k] : omax;
      fcnt += su[0][k];
      fent += su[1][k];
    }
    if (mmax) atomicMax(&imax[0], mmax);
    if (cmax) atomicMax(&imax[1], cmax);
    if (omax) atomicMax(&imax[2], omax);
    if (fcnt) atomicAdd(&fst[0], fcnt);
    if (fent) atomicAdd(&fst[1], fent);
  }
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// lAIR row of one C point per wave: N_i = strong F neighbours (sorted),
// T = A[N_i,N_i]^T, solve T z = -A[i,N_i]^T by LU with partial pivoting;
// injection (z = 0, counted) if N_i is empty or a pivot is <= 1e-14 max|T|.
// Distance-two lAIR neighbourhood of C point i by one 64-lane wave: the
// strong F neighbours of i, then the strong F neighbours of those (paths
// through F points only), gathered into cand[0..CAP) (LDS), sorted and made
// unique.  Returns the size m (the sorted set is cand[0..m)); returns -1 if
// more than CAP candidates arise.  *s_cnt is an LDS counter.
constexpr int NB2_CAP = 1024;

__device__ int nbhd2(int64_t i, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                     const uint8_t* __restrict__ strong, const int8_t* __restrict__ cf, int32_t* cand, int* s_cnt) {
  const int lane = threadIdx.x;
  if (lane == 0) *s_cnt = 0;
  __syncthreads();
  for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64)
    if (strong[k] && !cf[ci[k]]) {
      const int pos = atomicAdd(s_cnt, 1);
      if (pos < NB2_CAP) cand[pos] = ci[k];
    }
  __syncthreads();
  const int m1 = min(*s_cnt, NB2_CAP);
  for (int t = 0; t < m1; ++t) {
    const int32_t j = cand[t];
    for (int64_t k = rp[j] + lane; k < rp[j + 1]; k += 64) {
      const int32_t c = ci[k];
      if (strong[k] && !cf[c] && c != (int32_t)i) {
        const int pos = atomicAdd(s_cnt, 1);
        if (pos < NB2_CAP) cand[pos] = c;
      }
    }
  }
  __syncthreads();
  const int tot = *s_cnt;
  if (tot > NB2_CAP) return -1;
  int S = 1;
  while (S < tot) S <<= 1;
  for (int k = tot + lane; k < S; k += 64) cand[k] = 0x7fffffff;
  __syncthreads();
  for (int kk = 2; kk <= S; kk <<= 1)
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int x = lane; x < S; x += 64) {
        const int y = x ^ jj;
        if (y > x) {
          const bool up = (x & kk) == 0;
          const int32_t a = cand[x], b = cand[y];
          if ((a > b) == up) { cand[x] = b; cand[y] = a; }
        }
      }
      __syncthreads();
    }
  // unique, in place: a chunk compares each entry with its predecessor in
  // the sorted order (the previous chunk's last entry is carried in a
  // register, since that chunk's writes may already have replaced it)
  int base = 0;
  int32_t carry = 0;
  for (int k0 = 0; k0 < tot; k0 += 64) {
    const int k = k0 + lane;
    const int32_t v = k < tot ? cand[k] : 0x7fffffff;
    int32_t pv = __shfl_up(v, 1, 64);
    if (lane == 0) pv = carry;
    const bool keep = k < tot && (k == 0 || v != pv);
    carry = __shfl(v, 63, 64);
    const unsigned long long mask = __ballot(keep);
    __syncthreads();
    if (keep) cand[base + __popcll(mask & ((1ull << lane) - 1ull))] = v;
    base += __popcll(mask);
    __syncthreads();
  }
  return base;
}

// Distance-two lAIR: per C point the R row length 1 + |N_i| (rcnt), |N_i|
// (mcnt, -1 if the gather overflowed) and the R A P candidate bound (row
// lengths of A over {i} and N_i, ccnt).
__global__ __launch_bounds__(64) void k_lair_count2(int64_t nc, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const uint8_t* __restrict__ strong,
                                                    const int8_t* __restrict__ cf, const int32_t* __restrict__ clist,
                                                    int32_t* __restrict__ rcnt, int32_t* __restrict__ mcnt,
                                                    int32_t* __restrict__ ccnt) {
  __shared__ int32_t cand[NB2_CAP];
  __shared__ int s_cnt;
  const int64_t ic = blockIdx.x;
  const int64_t i = clist[ic];
  const int m = nbhd2(i, rp, ci, strong, cf, cand, &s_cnt);
  int64_t c = 0;
  if (m > 0)
    for (int t = threadIdx.x; t < m; t += 64) c += rp[cand[t] + 1] - rp[cand[t]];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (threadIdx.x == 0) {
    c += rp[i + 1] - rp[i];
    rcnt[ic] = 1 + (m > 0 ? m : 0);
    mcnt[ic] = m;
    ccnt[ic] = c > 0x3fffffff ? 0x3fffffff : (int32_t)c;
  }
}

// T[c m + r] = A[N_r, N_c] for the m rows N (sorted, m <= 64): the entries
// of all m rows at once, a lane per entry (its row r from the prefix sums of
// the row lengths), the column's position in N by binary search.  T must be
// zero on entry; pre (m + 1 ints) and st0 (m offsets) are LDS scratch.
__device__ void gather_nn(int m, const int32_t* N, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ v, double* T, int* pre, int64_t* st0, int lane) {
  int len = 0;
  int64_t s0 = 0;
  if (lane < m) {
    const int64_t j = N[lane];
    s0 = rp[j];
    len = (int)(rp[j + 1] - s0);
  }
  int inc = len;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane < m) { pre[lane + 1] = inc; st0[lane] = s0; }
  if (lane == 0) pre[0] = 0;
  __syncthreads();
  const int tot = pre[m];
  for (int e = lane; e < tot; e += 64) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {   // the last row starting at or before e
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int64_t k = st0[lo] + (e - pre[lo]);
    const int32_t col = ci[k];
    int a = 0, b = m - 1, c = -1;
    while (a <= b) {
      const int mid = (a + b) >> 1;
      if (N[mid] == col) { c = mid; break; }
      if (N[mid] < col) a = mid + 1; else b = mid - 1;
    }
    if (c >= 0) T[c * m + lo] = v[k];
  }
  __syncthreads();
}

// z <- T^-1 z for the m x m matrix T in LDS (row r at T[r m]) and nrhs
// right-hand sides z[q zs + r]: LU with partial pivoting carried through the
// right-hand sides, then back substitution.  Pivot: the largest |T[r][k]|,
// r >= k, smallest row on ties; a pivot at or below 1e-14 of sc (the largest
// |T|) marks the system bad, and later steps divide by 1 (the caller
// discards the result).  Each elimination step runs a lane per (row,
// column or right-hand side) pair with the row multipliers in f (LDS, m
// entries); the back substitution goes by columns, a lane per (row,
// right-hand side).  One wave; every lane calls it and gets the same result.
__device__ bool lu_solve_wave(int m, double* T, double* z, int zs, int nrhs, double* f, double sc, int lane) {
  bool bad = false;
  for (int k = 0; k < m; ++k) {
    double best = -1.0;
    int bi = m;
    for (int r = k + lane; r < m; r += 64) {
      const double a = fabs(T[r * m + k]);
      if (a > best) { best = a; bi = r; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const int p = bi;
    if (fabs(T[p * m + k]) <= 1e-14 * sc) bad = true;
    if (p != k) {
      for (int c = lane; c < m; c += 64) {
        const double t = T[k * m + c]; T[k * m + c] = T[p * m + c]; T[p * m + c] = t;
      }
      for (int q = lane; q < nrhs; q += 64) {
        const double t = z[q * zs + k]; z[q * zs + k] = z[q * zs + p]; z[q * zs + p] = t;
      }
    }
    __syncthreads();
    const double pv = bad ? 1.0 : T[k * m + k];
    for (int r = k + 1 + lane; r < m; r += 64) f[r] = T[r * m + k] / pv;
    __syncthreads();
    const int w = m - k - 1, nc = w + nrhs;
    for (int t = lane; t < w * nc; t += 64) {
      const int r = k + 1 + t / nc, cc = t % nc;
      if (cc < w) {
        T[r * m + k + 1 + cc] -= f[r] * T[k * m + k + 1 + cc];
      } else {
        const int q = cc - w;
        z[q * zs + r] -= f[r] * z[q * zs + k];
      }
    }
    __syncthreads();
  }
  for (int c = m - 1; c >= 0; --c) {
    const double dc = bad ? 1.0 : T[c * m + c];
    for (int q = lane; q < nrhs; q += 64) z[q * zs + c] /= dc;
    __syncthreads();
    for (int t = lane; t < c * nrhs; t += 64) {
      const int r = t / nrhs, q = t % nrhs;
      z[q * zs + r] -= T[r * m + c] * z[q * zs + c];
    }
    __syncthreads();
  }
  return bad;
}

template <int MAXM, bool D2>
__global__ __launch_bounds__(64) void k_lair(int64_t nc, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                             const double* __restrict__ v, const uint8_t* __restrict__ strong,
                                             const int8_t* __restrict__ cf, const int32_t* __restrict__ clist,
                                             const int64_t* __restrict__ Rptr, int32_t* __restrict__ Rcol,
                                             double* __restrict__ Rval, unsigned long long* __restrict__ nfall) {
  __shared__ int32_t Nbuf[D2 ? NB2_CAP : MAXM];
  __shared__ double T[MAXM * MAXM];
  __shared__ double z[MAXM];
  __shared__ int s_m;
  __shared__ int s_pre[MAXM + 1];
  __shared__ int64_t s_st0[MAXM];
  __shared__ double s_f[MAXM];
  int32_t* N = Nbuf;
  const int64_t ic = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t i = clist[ic];
  if (lane == 0) s_m = 0;
  __syncthreads();
  int m;
  if (D2) {
    // distance two: the sorted neighbourhood, then the right-hand side
    // -A[i, N_i] (zero where row i has no entry)
    m = nbhd2(i, rp, ci, strong, cf, Nbuf, &s_m);
    if (m < 0) m = MAXM + 1;
    for (int t = lane; t < MAXM; t += 64) z[t] = 0.0;
    __syncthreads();
    if (m <= MAXM)
      for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) {
        const int32_t col = ci[k];
        int lo = 0, hi = m - 1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          if (N[mid] == col) { z[mid] = -v[k]; break; }
          if (N[mid] < col) lo = mid + 1; else hi = mid - 1;
        }
      }
    __syncthreads();
  } else {
    // gather N_i and the right-hand side in row order (columns are sorted)
    int base = 0;
    for (int64_t k0 = rp[i]; k0 < rp[i + 1]; k0 += 64) {
      int64_t k = k0 + lane;
      bool f = k < rp[i + 1] && strong[k] && !cf[ci[k]];
      unsigned long long mask = __ballot(f);
      int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
      if (f && pos < MAXM) { N[pos] = ci[k]; z[pos] = -v[k]; }
      base += __popcll(mask);
    }
    m = base;
  }
  const int64_t out = Rptr[ic];
  if (m == 0 || m > MAXM) {
    // m > MAXM cannot occur: the host picks MAXM >= max |N_i|
    if (lane == 0) {
      Rcol[out] = (int32_t)i;
      Rval[out] = 1.0;
      atomicAdd(nfall, 1ull);
    }
    return;
  }
  for (int k = lane; k < m * m; k += 64) T[k] = 0.0;
  __syncthreads();
  // T[c][r] = A[N_r, N_c]
  gather_nn(m, N, rp, ci, v, T, s_pre, s_st0, lane);
  double sc = 0.0;
  for (int k = lane; k < m * m; k += 64) sc = fmax(sc, fabs(T[k]));
  sc = wave_max(sc);
  const bool bad = lu_solve_wave(m, T, z, MAXM, 1, s_f, sc, lane);
  // row in increasing column order: N is sorted, the C point itself is not in N
  int ins = 0;
  for (int r = lane; r < m; r += 64) ins += N[r] < i;
  for (int o = 32; o > 0; o >>= 1) ins += __shfl_xor(ins, o, 64);
  for (int r = lane; r < m; r += 64) {
    int pos = r < ins ? r : r + 1;
    Rcol[out + pos] = N[r];
    Rval[out + pos] = bad ? 0.0 : z[r];
  }
  if (lane == 0) {
    Rcol[out + ins] = (int32_t)i;
    Rval[out + ins] = 1.0;
    if (bad) atomicAdd(nfall, 1ull);
  }
}

// Block AIR lAIR rows (level 0): one wave per C block, rows i0 .. i0 + b - 1.
// Every row of a block holds the same off-diagonal blocks in full, so N (the
// rows of the strong F blocks) and its order come from each row alike; the
// b right-hand sides -A[i0 + r, N]^T are gathered in that order, T =
// A[N, N]^T is factored once by LU with partial pivoting, and the
// right-hand sides are carried through the same eliminations and back
// substitutions as in k_lair (lu_solve_wave), so each row gets the values
// k_lair would give it.  *err is set if the rows of a block disagree on |N|.
constexpr int LB_BMAX = 10;

template <int MAXM>
__global__ __launch_bounds__(64) void k_lair_blk(int64_t ncb, int b, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                 const uint8_t* __restrict__ strong, const int8_t* __restrict__ cf,
                                                 const int32_t* __restrict__ clist, const int64_t* __restrict__ Rptr,
                                                 int32_t* __restrict__ Rcol, double* __restrict__ Rval,
                                                 unsigned long long* __restrict__ nfall, int* __restrict__ err) {
  __shared__ int32_t N[MAXM];
  __shared__ double T[MAXM * MAXM];
  __shared__ double z[LB_BMAX * MAXM];
  __shared__ int s_pre[MAXM + 1];
  __shared__ int64_t s_st0[MAXM];
  __shared__ double s_f[MAXM];
  const int64_t kb = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t i0 = clist[kb * b];
  int m = 0;
  for (int q = 0; q < b; ++q) {
    const int64_t i = i0 + q;
    int base = 0;
    for (int64_t k0 = rp[i]; k0 < rp[i + 1]; k0 += 64) {
      const int64_t k = k0 + lane;
      const bool f = k < rp[i + 1] && strong[k] && !cf[ci[k]];
      const unsigned long long mask = __ballot(f);
      const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
      if (f && pos < MAXM) {
        if (q == 0) N[pos] = ci[k];
        z[q * MAXM + pos] = -v[k];
      }
      base += __popcll(mask);
    }
    if (q == 0) m = base;
    else if (base != m && lane == 0) atomicOr(err, 1);
  }
  __syncthreads();
  if (m == 0 || m > MAXM) {
    // m > MAXM cannot occur: the host picks MAXM >= max |N|
    if (lane < b) {
      const int64_t out = Rptr[kb * b + lane];
      Rcol[out] = (int32_t)(i0 + lane);
      Rval[out] = 1.0;
    }
    if (lane == 0) atomicAdd(nfall, (unsigned long long)b);
    return;
  }
  for (int k = lane; k < m * m; k += 64) T[k] = 0.0;
  __syncthreads();
  // T[c][r] = A[N_r, N_c]
  gather_nn(m, N, rp, ci, v, T, s_pre, s_st0, lane);
  double sc = 0.0;
  for (int k = lane; k < m * m; k += 64) sc = fmax(sc, fabs(T[k]));
  sc = wave_max(sc);
  const bool bad = lu_solve_wave(m, T, z, MAXM, b, s_f, sc, lane);
  // rows in increasing column order: N is sorted and holds no row of the block
  int ins = 0;
  for (int r = lane; r < m; r += 64) ins += N[r] < i0;
  for (int o = 32; o > 0; o >>= 1) ins += __shfl_xor(ins, o, 64);
  for (int q = 0; q < b; ++q) {
    const int64_t out = Rptr[kb * b + q];
    for (int r = lane; r < m; r += 64) {
      const int pos = r < ins ? r : r + 1;
      Rcol[out + pos] = N[r];
      Rval[out + pos] = bad ? 0.0 : z[q * MAXM + r];
    }
    if (lane == 0) {
      Rcol[out + ins] = (int32_t)(i0 + q);
      Rval[out + ins] = 1.0;
    }
  }
  if (bad && lane == 0) atomicAdd(nfall, (unsigned long long)b);
}

// R A P per coarse row with an LDS open-addressing hash on the coarse
// column (HS >= candidates, so it never overflows).  NUMERIC = false counts
// the distinct columns; NUMERIC = true accumulates, sorts and writes.
template <int HS, bool NUMERIC>
__global__ __launch_bounds__(64) void k_rap(int64_t nc, const int64_t* __restrict__ Rptr, const int32_t* __restrict__ Rcol,
                                            const double* __restrict__ Rval, const int64_t* __restrict__ rp,
                                            const int32_t* __restrict__ ci, const double* __restrict__ v,
                                            const int32_t* __restrict__ pcol, int32_t* __restrict__ cnt,
                                            const int64_t* __restrict__ cptr, int32_t* __restrict__ ccol,
                                            double* __restrict__ cval) {
  __shared__ int32_t key[HS];
  __shared__ double val[NUMERIC ? HS : 1];
  __shared__ int s_cnt;
  __shared__ int s_pre[65];
  __shared__ int64_t s_st[64];
  __shared__ double s_rv[64];
  const int64_t ic = blockIdx.x;
  const int lane = threadIdx.x;
  for (int k = lane; k < HS; k += 64) {
    key[k] = -1;
    if (NUMERIC) val[k] = 0.0;
  }
  if (lane == 0) s_cnt = 0;
  __syncthreads();
  // the rows of A named by up to 64 entries of the R row at once: a lane per
  // (R entry, A entry) pair, the R entry from the prefix sums of the row
  // lengths
  const int64_t r0 = Rptr[ic], r1 = Rptr[ic + 1];
  for (int64_t c0 = r0; c0 < r1; c0 += 64) {
    const int cl = (int)(r1 - c0 < 64 ? r1 - c0 : 64);
    int len = 0;
    int64_t s0 = 0;
    double rv0 = 0.0;
    if (lane < cl) {
      const int32_t j = Rcol[c0 + lane];
      s0 = rp[j];
      len = (int)(rp[j + 1] - s0);
      if (NUMERIC) rv0 = Rval[c0 + lane];
    }
    int inc = len;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane < cl) { s_pre[lane + 1] = inc; s_st[lane] = s0; s_rv[lane] = rv0; }
    if (lane == 0) s_pre[0] = 0;
    __syncthreads();
    const int ne = s_pre[cl];
    for (int e = lane; e < ne; e += 64) {
      int lo = 0, hi = cl - 1;
      while (lo < hi) {   // the last R entry whose row starts at or before e
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
      }
      const int64_t k = s_st[lo] + (e - s_pre[lo]);
      const int32_t c = pcol[ci[k]];
      if (c < 0) continue;
      uint32_t h = ((uint32_t)c * 2654435761u) & (HS - 1);
      while (true) {
        const int32_t prev = atomicCAS(&key[h], -1, c);
        if (prev == -1 || prev == c) {
          if (prev == -1) atomicAdd(&s_cnt, 1);
          if (NUMERIC) atomicAdd(&val[h], s_rv[lo] * v[k]);
          break;
        }
        h = (h + 1) & (HS - 1);
      }
    }
    __syncthreads();
  }
  if (!NUMERIC) {
    if (lane == 0) cnt[ic] = s_cnt;
    return;
  }
  // compact to the front in place: one wave reads a chunk before writing it,
  // and every write position is <= the positions still to be read
  const int tot = s_cnt;
  int32_t* ck = key;
  double* cv = val;
  int base = 0;
  for (int k0 = 0; k0 < HS; k0 += 64) {
    int k = k0 + lane;
    int32_t kk = key[k];
    double vv = val[k];
    bool occ = kk >= 0;
    unsigned long long mask = __ballot(occ);
    int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
    __syncthreads();
    if (occ) { ck[pos] = kk; cv[pos] = vv; }
    base += __popcll(mask);
    __syncthreads();
  }
  const int64_t o = cptr[ic];
  if (tot <= 64) {
    // at most one column per lane: its place in the row is the number of
    // smaller columns (the columns are distinct)
    if (lane < tot) {
      const int32_t my = ck[lane];
      int r = 0;
      for (int j = 0; j < tot; ++j) r += ck[j] < my;
      ccol[o + r] = my;
      cval[o + r] = cv[lane];
    }
    return;
  }
  int S = 1;
  while (S < tot) S <<= 1;
  for (int k = tot + lane; k < S; k += 64) ck[k] = 0x7fffffff;
  __syncthreads();
  // bitonic sort by column
  for (int kk = 2; kk <= S; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int x = lane; x < S; x += 64) {
        int y = x ^ jj;
        if (y > x) {
          bool up = (x & kk) == 0;
          int32_t a = ck[x], b = ck[y];
          if ((a > b) == up) {
            ck[x] = b; ck[y] = a;
            double t = cv[x]; cv[x] = cv[y]; cv[y] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int k = lane; k < tot; k += 64) {
    ccol[o + k] = ck[k];
    cval[o + k] = cv[k];
  }
}

// R A P for the b coarse rows of a block AIR C block (level 0), one wave
// per block: the rows of R of a block have the same length and hold the
// same neighbourhood columns at the same positions, with each row's own
// column at one common position.  A row of the neighbourhood is read once
// for all b coarse rows (k_rap reads it once per row); the own rows are
// read once each.  One LDS hash on the coarse column holds b sums and a
// mask of the rows that reached the column, so every coarse row gets the
// columns k_rap gives it, and the same sums up to the order of additions.
// NUMERIC = false counts the columns of each row; NUMERIC = true sums,
// sorts by column and writes the b rows.
template <int HS, bool NUMERIC, int B>
__global__ __launch_bounds__(64) void k_rap_blk(int64_t ncb, const int64_t* __restrict__ Rptr,
                                                const int32_t* __restrict__ Rcol, const double* __restrict__ Rval,
                                                const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                const double* __restrict__ v, const int32_t* __restrict__ pcol,
                                                const int32_t* __restrict__ clist, int32_t* __restrict__ cnt,
                                                const int64_t* __restrict__ cptr, int32_t* __restrict__ ccol,
                                                double* __restrict__ cval) {
  __shared__ int32_t key[HS];
  __shared__ uint32_t tch[HS];
  __shared__ double val[NUMERIC ? HS * B : 1];
  __shared__ int32_t sidx[NUMERIC ? HS : 1];
  __shared__ int s_cnt;
  __shared__ int s_pre[65];
  __shared__ int64_t s_st[64];
  __shared__ double s_rv[NUMERIC ? 64 * B : 1];
  const int64_t r0 = (int64_t)blockIdx.x * B;
  const int lane = threadIdx.x;
  for (int k = lane; k < HS; k += 64) {
    key[k] = -1;
    tch[k] = 0u;
    if (NUMERIC)
      for (int q = 0; q < B; ++q) val[k * B + q] = 0.0;
  }
  if (lane == 0) s_cnt = 0;
  __syncthreads();
  const int64_t i0 = clist[r0];
  const int64_t base0 = Rptr[r0];
  const int len = (int)(Rptr[r0 + 1] - base0);
  // the neighbourhood rows named by up to 64 R positions at once (a lane per
  // (position, entry) pair, the position from the prefix sums of the row
  // lengths), each with the b coefficients of the block's R rows; then the
  // block's own rows i0 + q, row q with the coefficient of coarse row q only
  int tpos = -1;
  for (int t0 = 0; t0 < len; t0 += 64) {
    const int cl = len - t0 < 64 ? len - t0 : 64;
    int rl = 0;
    int64_t s0 = 0;
    if (lane < cl) {
      const int32_t j = Rcol[base0 + t0 + lane];
      if (j == (int32_t)i0) {
        tpos = t0 + lane;
      } else {
        s0 = rp[j];
        rl = (int)(rp[j + 1] - s0);
      }
      if (NUMERIC)
#pragma unroll
        for (int u = 0; u < B; ++u) s_rv[lane * B + u] = Rval[Rptr[r0 + u] + t0 + lane];
    }
    int inc = rl;
    for (int o = 1; o < 64; o <<= 1) {
      const int tt = __shfl_up(inc, o, 64);
      if (lane >= o) inc += tt;
    }
    if (lane < cl) { s_pre[lane + 1] = inc; s_st[lane] = s0; }
    if (lane == 0) s_pre[0] = 0;
    __syncthreads();
    const int ne = s_pre[cl];
    for (int e = lane; e < ne; e += 64) {
      int lo = 0, hi = cl - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
      }
      const int64_t k = s_st[lo] + (e - s_pre[lo]);
      const int32_t c = pcol[ci[k]];
      if (c < 0) continue;
      uint32_t h = ((uint32_t)c * 2654435761u) & (HS - 1);
      while (true) {
        const int32_t prev = atomicCAS(&key[h], -1, c);
        if (prev == -1 || prev == c) {
          if (prev == -1) atomicAdd(&s_cnt, 1);
          atomicOr(&tch[h], (1u << B) - 1u);
          if (NUMERIC)
#pragma unroll
            for (int u = 0; u < B; ++u) atomicAdd(&val[h * B + u], s_rv[lo * B + u] * v[k]);
          break;
        }
        h = (h + 1) & (HS - 1);
      }
    }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) tpos = max(tpos, __shfl_xor(tpos, o, 64));
  if (tpos >= 0) {
    int rl = 0;
    int64_t s0 = 0;
    if (lane < B) {
      s0 = rp[i0 + lane];
      rl = (int)(rp[i0 + lane + 1] - s0);
      if (NUMERIC) s_rv[lane] = Rval[Rptr[r0 + lane] + tpos];
    }
    int inc = rl;
    for (int o = 1; o < 64; o <<= 1) {
      const int tt = __shfl_up(inc, o, 64);
      if (lane >= o) inc += tt;
    }
    if (lane < B) { s_pre[lane + 1] = inc; s_st[lane] = s0; }
    if (lane == 0) s_pre[0] = 0;
    __syncthreads();
    const int ne = s_pre[B];
    for (int e = lane; e < ne; e += 64) {
      int q = 0;
      while (q + 1 < B && s_pre[q + 1] <= e) ++q;
      const int64_t k = s_st[q] + (e - s_pre[q]);
      const int32_t c = pcol[ci[k]];
      if (c < 0) continue;
      uint32_t h = ((uint32_t)c * 2654435761u) & (HS - 1);
      while (true) {
        const int32_t prev = atomicCAS(&key[h], -1, c);
        if (prev == -1 || prev == c) {
          if (prev == -1) atomicAdd(&s_cnt, 1);
          atomicOr(&tch[h], 1u << q);
          if (NUMERIC) atomicAdd(&val[h * B + q], s_rv[q] * v[k]);
          break;
        }
        h = (h + 1) & (HS - 1);
      }
    }
  }
  __syncthreads();
  if (!NUMERIC) {
    int c[B];
#pragma unroll
    for (int q = 0; q < B; ++q) c[q] = 0;
    for (int k = lane; k < HS; k += 64)
#pragma unroll
      for (int q = 0; q < B; ++q) c[q] += (tch[k] >> q) & 1u;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      for (int o = 32; o > 0; o >>= 1) c[q] += __shfl_xor(c[q], o, 64);
      if (lane == 0) cnt[r0 + q] = c[q];
    }
    return;
  }
  // occupied slots to the front as (column, slot) pairs: one wave reads a
  // chunk before writing it, and every write position is <= the positions
  // still to be read
  const int tot = s_cnt;
  int base = 0;
  for (int k0 = 0; k0 < HS; k0 += 64) {
    const int k = k0 + lane;
    const int32_t kk = key[k];
    const bool occ = kk >= 0;
    const unsigned long long mask = __ballot(occ);
    const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
    __syncthreads();
    if (occ) { key[pos] = kk; sidx[pos] = k; }
    base += __popcll(mask);
    __syncthreads();
  }
  if (tot <= 64) {
    // at most one column per lane: its place in coarse row q is the number
    // of smaller columns that row q reached (the columns are distinct)
    if (lane < tot) {
      const int32_t my = key[lane];
      const int sl = sidx[lane];
      const uint32_t mb = tch[sl];
      int r[B];
#pragma unroll
      for (int q = 0; q < B; ++q) r[q] = 0;
      for (int j = 0; j < tot; ++j)
        if (key[j] < my) {
          const uint32_t bj = tch[sidx[j]];
#pragma unroll
          for (int q = 0; q < B; ++q) r[q] += (bj >> q) & 1u;
        }
#pragma unroll
      for (int q = 0; q < B; ++q)
        if ((mb >> q) & 1u) {
          const int64_t o = cptr[r0 + q];
          ccol[o + r[q]] = my;
          cval[o + r[q]] = val[sl * B + q];
        }
    }
    return;
  }
  int S = 1;
  while (S < tot) S <<= 1;
  for (int k = tot + lane; k < S; k += 64) key[k] = 0x7fffffff;
  __syncthreads();
  for (int kk = 2; kk <= S; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int x = lane; x < S; x += 64) {
        const int y = x ^ jj;
        if (y > x) {
          const bool up = (x & kk) == 0;
          const int32_t a = key[x], bb = key[y];
          if ((a > bb) == up) {
            key[x] = bb; key[y] = a;
            const int32_t t = sidx[x]; sidx[x] = sidx[y]; sidx[y] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int q = 0; q < B; ++q) {
    const int64_t o = cptr[r0 + q];
    int wbase = 0;
    for (int k0 = 0; k0 < tot; k0 += 64) {
      const int k = k0 + lane;
      const int sl = k < tot ? sidx[k] : 0;
      const bool has = k < tot && ((tch[sl] >> q) & 1u);
      const unsigned long long mask = __ballot(has);
      if (has) {
        const int pos = wbase + __popcll(mask & ((1ull << lane) - 1ull));
        ccol[o + pos] = key[k];
        cval[o + pos] = val[sl * B + q];
      }
      wbase += __popcll(mask);
    }
  }
}

// Diagonal of a CSR matrix (0 where a row has no diagonal entry), PG lanes
// per row.
__global__ __launch_bounds__(256) void k_diag(int64_t n, const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ ci, const double* __restrict__ v,
                                              double* __restrict__ d, float* __restrict__ d32) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gid / PG;
  const int g = (int)(gid % PG);
  if (i >= n) return;
  double x = 0.0;
  int hit = 0;
  for (int64_t k = rp[i] + g; k < rp[i + 1]; k += PG)
    if (ci[k] == i) { x = v[k]; hit = 1; break; }
  // the row holds at most one diagonal entry: its lane passes it on
  for (int o = PG / 2; o > 0; o >>= 1) {
    const double ox = __shfl_xor(x, o, PG);
    const int oh = __shfl_xor(hit, o, PG);
    if (oh) { x = ox; hit = 1; }
  }
  if (g != 0) return;
  d[i] = x;
  if (d32) d32[i] = (float)x;
}

// Stored values of the listed level-0 rows in the off-diagonal facet-block
// layout (B per off-diagonal block of the row's block row), one atomic per
// block.
__global__ __launch_bounds__(256) void k_list_vals(int64_t nl, const int32_t* __restrict__ list,
                                                   const int64_t* __restrict__ optr, int B,
                                                   unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[4];
  unsigned long long acc = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nl; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t R = list[k] / B;
    acc += (unsigned long long)(optr[R + 1] - optr[R]) * (unsigned long long)B;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = red[0] + red[1] + red[2] + red[3];
    if (t) atomicAdd(out, t);
  }
}

__global__ void k_cast32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// Dense copy of the coarsest matrix.
__global__ void k_dense(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                        const double* __restrict__ v, double* __restrict__ M) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) M[i * n + ci[k]] = v[k];
}

// Gauss-Jordan with partial pivoting on [M | Inv] over many workgroups, one
// column c per pair of launches (within one workgroup the n^3 updates of a
// few hundred rows take tens of milliseconds on one compute unit).
// k_gj_pivot (one workgroup): pivot search in column c (largest |M[r][c]|,
// r >= c, smallest row on ties), row swap,
// scaling of the pivot row, and the multipliers f[r] = M[r][c] (f[c] = 0).
__global__ __launch_bounds__(1024) void k_gj_pivot(int n, int c, double* __restrict__ M, double* __restrict__ Inv,
                                                   double* __restrict__ f, int* __restrict__ err) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ int s_p;
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int r = c + t; r < n; r += blockDim.x) {
    const double a = fabs(M[(int64_t)r * n + c]);
    if (a > best) { best = a; bi = r; }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s && (sv[t + s] > sv[t] || (sv[t + s] == sv[t] && si[t + s] < si[t]))) {
      sv[t] = sv[t + s];
      si[t] = si[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    s_p = si[0];
    if (!(sv[0] > 0.0)) atomicOr(err, 1);
  }
  __syncthreads();
  const int p = s_p;
  if (p != c)
    for (int j = t; j < n; j += blockDim.x) {
      double x = M[(int64_t)c * n + j]; M[(int64_t)c * n + j] = M[(int64_t)p * n + j]; M[(int64_t)p * n + j] = x;
      x = Inv[(int64_t)c * n + j]; Inv[(int64_t)c * n + j] = Inv[(int64_t)p * n + j]; Inv[(int64_t)p * n + j] = x;
    }
  __syncthreads();
  double d = M[(int64_t)c * n + c];
  if (d == 0.0) d = 1.0;
  __syncthreads();
  for (int j = t; j < n; j += blockDim.x) {
    M[(int64_t)c * n + j] /= d;
    Inv[(int64_t)c * n + j] /= d;
  }
  for (int r = t; r < n; r += blockDim.x) f[r] = r == c ? 0.0 : M[(int64_t)r * n + c];
}

// Elimination of column c from every other row, a thread per entry of
// [M | Inv]: M[r][j] -= f[r] M[c][j] (j > c; M[r][c] = 0; the columns left
// of c hold zeros in the pivot row), Inv[r][j] -= f[r] Inv[c][j].
__global__ __launch_bounds__(256) void k_gj_update(int n, int c, double* __restrict__ M, double* __restrict__ Inv,
                                                   const double* __restrict__ f) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t w = 2 * (int64_t)n;
  if (idx >= (int64_t)n * w) return;
  const int r = (int)(idx / w), jj = (int)(idx % w);
  if (r == c) return;
  const double fr = f[r];
  if (jj < n) {
    if (jj > c) M[(int64_t)r * n + jj] -= fr * M[(int64_t)c * n + jj];
    else if (jj == c) M[(int64_t)r * n + c] = 0.0;
  } else {
    const int j = jj - n;
    Inv[(int64_t)r * n + j] -= fr * Inv[(int64_t)c * n + j];
  }
}

// Identity of order n.
__global__ void k_eye(int n, double* __restrict__ Inv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < (int64_t)n * n) Inv[k] = (k / n == k % n) ? 1.0 : 0.0;
}

// Inverse of a dense matrix of order n <= 64 by Gauss-Jordan elimination
// with partial pivoting on the augmented matrix [A | I], held entirely in
// LDS (64 x 128 doubles).
constexpr int INV_GJ_MAX = 64;

__global__ __launch_bounds__(256) void k_inv_gj(int n, const double* __restrict__ M, double* __restrict__ Inv,
                                                int* __restrict__ err) {
  __shared__ double A[INV_GJ_MAX * 2 * INV_GJ_MAX];
  __shared__ double f[INV_GJ_MAX];
  __shared__ int s_p;
  const int t = threadIdx.x;
  const int W = 2 * n;
  for (int idx = t; idx < n * W; idx += blockDim.x) {
    int r = idx / W, c = idx % W;
    A[idx] = c < n ? M[r * n + c] : (c - n == r ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (t < 64) {
      double best = -1.0;
      int bi = n;
      int r = k + t;
      if (r < n) { best = fabs(A[r * W + k]); bi = r; }
      for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (t == 0) {
        s_p = bi;
        if (!(best > 0.0)) atomicOr(err, 1);
      }
    }
    __syncthreads();
    const int p = s_p;
    if (p != k)
      for (int c = t; c < W; c += blockDim.x) {
        double x = A[k * W + c]; A[k * W + c] = A[p * W + c]; A[p * W + c] = x;
      }
    __syncthreads();
    const double d = A[k * W + k] != 0.0 ? A[k * W + k] : 1.0;
    if (t < n) f[t] = t == k ? 0.0 : A[t * W + k];
    __syncthreads();
    for (int c = t; c < W; c += blockDim.x) A[k * W + c] /= d;
    __syncthreads();
    for (int idx = t; idx < n * W; idx += blockDim.x) {
      int r = idx / W, c = idx % W;
      if (r != k) A[idx] -= f[r] * A[k * W + c];
    }
    __syncthreads();
  }
  for (int idx = t; idx < n * n; idx += blockDim.x) {
    int r = idx / n, c = idx % n;
    Inv[idx] = A[r * W + n + c];
  }
}

// Inverse of a small dense matrix held in LDS (n <= 128): LU with partial
// pivoting (largest magnitude, smallest row on ties), then one column of
// the inverse per thread by forward and back substitution.
constexpr int INV_LDS_MAX = 128;

__global__ __launch_bounds__(1024) void k_inv_lds(int n, const double* __restrict__ M, double* __restrict__ Inv,
                                                  int* __restrict__ err) {
  __shared__ double A[INV_LDS_MAX * INV_LDS_MAX];
  __shared__ int piv[INV_LDS_MAX];
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  for (int k = t; k < n * n; k += NT) A[k] = M[k];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (t < 64) {
      double best = -1.0;
      int bi = n;
      for (int r = k + t; r < n; r += 64) {
        double a = fabs(A[r * n + k]);
        if (a > best) { best = a; bi = r; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (t == 0) {
        piv[k] = bi;
        if (!(best > 0.0)) atomicOr(err, 1);
      }
    }
    __syncthreads();
    const int p = piv[k];
    if (p != k)
      for (int c = t; c < n; c += NT) {
        double x = A[k * n + c]; A[k * n + c] = A[p * n + c]; A[p * n + c] = x;
      }
    __syncthreads();
    const double d = A[k * n + k] != 0.0 ? A[k * n + k] : 1.0;
    for (int r = k + 1 + t; r < n; r += NT) A[r * n + k] /= d;
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = t; idx < m * m; idx += NT) {
      int r = k + 1 + idx / m, c = k + 1 + idx % m;
      A[r * n + c] -= A[r * n + k] * A[k * n + c];
    }
    __syncthreads();
  }
  for (int j = t; j < n; j += NT) {
    double x[INV_LDS_MAX];
    for (int r = 0; r < n; ++r) x[r] = (r == j) ? 1.0 : 0.0;
    for (int k = 0; k < n; ++k) {
      int p = piv[k];
      double tmp = x[k]; x[k] = x[p]; x[p] = tmp;
    }
    for (int r = 1; r < n; ++r) {
      double v = x[r];
      for (int k = 0; k < r; ++k) v -= A[r * n + k] * x[k];
      x[r] = v;
    }
    for (int r = n - 1; r >= 0; --r) {
      double v = x[r];
      for (int k = r + 1; k < n; ++k) v -= A[r * n + k] * x[k];
      x[r] = v / A[r * n + r];
    }
    for (int r = 0; r < n; ++r) Inv[(int64_t)r * n + j] = x[r];
  }
}

// CSR transpose: counts, offsets, scatter with an atomic cursor, then each
// row sorted by column so the result does not depend on scheduling.
__global__ void k_tcount(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         int32_t* __restrict__ cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) atomicAdd(&cnt[ci[k]], 1);
}

__global__ void k_tscatter(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, const int64_t* __restrict__ tp, int32_t* __restrict__ cur,
                           int32_t* __restrict__ tc, double* __restrict__ tv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
    int32_t j = ci[k];
    int64_t pos = tp[j] + atomicAdd(&cur[j], 1);
    tc[pos] = (int32_t)i;
    if (tv) tv[pos] = v ? v[k] : 1.0;
  }
}

__global__ void k_rowsort(int64_t n, const int64_t* __restrict__ tp, int32_t* __restrict__ tc, double* __restrict__ tv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t a = tp[i] + 1; a < tp[i + 1]; ++a) {
    int32_t kc = tc[a];
    double kv = tv ? tv[a] : 0.0;
    int64_t b = a - 1;
    while (b >= tp[i] && tc[b] > kc) {
      tc[b + 1] = tc[b];
      if (tv) tv[b + 1] = tv[b];
      --b;
    }
    tc[b + 1] = kc;
    if (tv) tv[b + 1] = kv;
  }
}

// P as CSR: one entry (pcol[i], 1) per fine point with pcol >= 0.
__global__ void k_p_rowcnt(int64_t n, const int32_t* __restrict__ pcol, int32_t* __restrict__ cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = pcol[i] >= 0;
}

__global__ void k_p_fill(int64_t n, const int32_t* __restrict__ pcol, const int64_t* __restrict__ pp,
                         int32_t* __restrict__ pc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && pcol[i] >= 0) pc[pp[i]] = pcol[i];
}

static inline dim3 g1(int64_t n, int t = 256) { return dim3((unsigned)cdiv(std::max<int64_t>(n, 1), t)); }
// Capped grid for the grid-stride kernels with PG lanes per row (256 threads).
static inline dim3 grows(int64_t n) {
  return dim3((unsigned)std::min<int64_t>(cdiv(std::max<int64_t>(n, 1), 256 / PG), 2048));
}

// Transposed level-0 operator in the facet-block layout: block row I, slot
// s (column block J) receives the transpose of block (J, I), found in the
// slots of block row J; a slot without a transposed slot sets *bad.
__global__ void k_fb_transpose(int64_t nbr, int B, const int64_t* __restrict__ optr,
                               const int32_t* __restrict__ ocol, const double* __restrict__ ov,
                               double* __restrict__ otv, int* __restrict__ bad) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nbr) return;
  const int64_t oi = optr[I];
  const int64_t leni = (optr[I + 1] - oi) * B;
  for (int64_t s = oi; s < optr[I + 1]; ++s) {
    const int32_t J = ocol[s];
    const int64_t oj = optr[J];
    int64_t t = -1;
    for (int64_t q = oj; q < optr[J + 1]; ++q)
      if (ocol[q] == (int32_t)I) { t = q; break; }
    if (t < 0) { *bad = 1; continue; }
    const int64_t lenj = (optr[J + 1] - oj) * B;
    const double* __restrict__ src = ov + oj * B * B + (t - oj) * B;
    double* __restrict__ dst = otv + oi * B * B + (s - oi) * B;
    for (int m = 0; m < B; ++m)
      for (int c = 0; c < B; ++c) dst[m * leni + c] = src[c * lenj + m];
  }
}

static ah_status transpose(int64_t nrow, int64_t ncol, const int64_t* rp, const int32_t* ci, const double* v,
                           int64_t nnz, Arena& ar, Arena& tmp, hipStream_t st, int64_t** tp, int32_t** tc,
                           double** tv) {
  int32_t* cnt = nullptr;
  AH_TRY(tmp.get(&cnt, ncol + 1));
  AH_HIP(hipMemsetAsync(cnt, 0, (ncol + 1) * sizeof(int32_t), st));
  hipLaunchKernelGGL(k_tcount, g1(nrow), dim3(256), 0, st, nrow, rp, ci, cnt);
  AH_LAUNCHED();
  AH_TRY(ar.get(tp, ncol + 1));
  AH_TRY(scan_i32_to_i64(cnt, *tp, ncol, st, tmp));
  AH_TRY(ar.get(tc, nnz));
  if (tv) AH_TRY(ar.get(tv, nnz));
  AH_HIP(hipMemsetAsync(cnt, 0, (ncol + 1) * sizeof(int32_t), st));
  hipLaunchKernelGGL(k_tscatter, g1(nrow), dim3(256), 0, st, nrow, rp, ci, v, *tp, cnt, *tc, tv ? *tv : nullptr);
  AH_LAUNCHED();
  hipLaunchKernelGGL(k_rowsort, g1(ncol), dim3(256), 0, st, ncol, *tp, *tc, tv ? *tv : nullptr);
  AH_LAUNCHED();
  return AH_OK;
}

// out[0] = max(out[0], max of a[0..n)): grid-stride, one atomic per block.
__global__ __launch_bounds__(256) void k_max_i32(int64_t n, const int32_t* __restrict__ a, int* __restrict__ out) {
  __shared__ int red[4];
  int m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = a[i] > m ? a[i] : m;
  for (int o = 32; o > 0; o >>= 1) {
    const int q = __shfl_xor(m, o, 64);
    m = q > m ? q : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int b = max(max(red[0], red[1]), max(red[2], red[3]));
    if (b) atomicMax(out, b);
  }
}

// Block AIR on a scaled level 0 (facet blocks of b rows; the facet-block
// copy holds block row I as [b][nob][b] values from optr[I] b^2 on).
// Block weight of every off-diagonal block slot: w = max |a_ij| over the
// block.  SG lanes per block row, a lane per slot.
__global__ __launch_bounds__(256) void k_block_weights(int64_t nbr, int b, const int64_t* __restrict__ optr,
                                                       const double* __restrict__ oval, double* __restrict__ w) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t I = gid / SG;
  const int g = (int)(gid % SG);
  if (I >= nbr) return;
  const int64_t s0 = optr[I];
  const int nob = (int)(optr[I + 1] - s0);
  const double* row = oval + s0 * b * b;
  for (int s = g; s < nob; s += SG) {
    double m = 0.0;
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c) m = fmax(m, fabs(row[((int64_t)r * nob + s) * b + c]));
    w[s0 + s] = m;
  }
}

// Every row of a block takes its block's PMIS state.
__global__ void k_block_expand(int64_t n, int b, const int8_t* __restrict__ sb, int8_t* __restrict__ state) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) state[i] = sb[i / b];
}

// Scalar strong mask of the level-0 CSR from the block marks: entry (i, j)
// is strong when blocks i/b != j/b are joined by a strong block slot (the
// slots of a block row are sorted by column).  PG lanes per row.  The
// scaled row holds the off-diagonal blocks in column order, b entries
// each, and the single diagonal entry of the identity diagonal block, so
// entry t is in slot t / b before the diagonal and (t - 1) / b after it:
// that slot is tried first, then a binary search.
__global__ __launch_bounds__(256) void k_block_mask(int64_t n, int b, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const int64_t* __restrict__ optr,
                                                    const int32_t* __restrict__ ocol,
                                                    const uint8_t* __restrict__ sb, uint8_t* __restrict__ strong) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gid / PG;
  const int g = (int)(gid % PG);
  if (i >= n) return;
  const int64_t I = i / b, lo0 = optr[I], hi0 = optr[I + 1] - 1;
  const int64_t r0 = rp[i];
  for (int64_t k = r0 + g; k < rp[i + 1]; k += PG) {
    const int32_t J = ci[k] / b;
    uint8_t f = 0;
    const int64_t q = lo0 + (J > I ? (k - r0 - 1) / b : (k - r0) / b);
    if (J != I && q >= lo0 && q <= hi0 && ocol[q] == J) {
      f = sb[q];
    } else if (J != I) {
      int64_t lo = lo0, hi = hi0;
      while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ocol[mid] == J) { f = sb[mid]; break; }
        if (ocol[mid] < J) lo = mid + 1; else hi = mid - 1;
      }
    }
    strong[k] = f;
  }
}

// Block one-point interpolation: an F block takes the strongest strong C
// block (largest w, ties to the smallest block index, within relative
// 1e-12 of the maximum), and row m of it interpolates from row m of that
// block: pcol[I b + m] = cidx[J b + m]; -1 without a strong C block.
__global__ void k_block_pcol(int64_t nbr, int b, const int64_t* __restrict__ optr, const int32_t* __restrict__ ocol,
                             const double* __restrict__ w, const uint8_t* __restrict__ sb,
                             const int8_t* __restrict__ cf, const int64_t* __restrict__ cidx,
                             int32_t* __restrict__ pcol) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nbr || cf[I * b]) return;
  double mx = -1.0;
  for (int64_t q = optr[I]; q < optr[I + 1]; ++q)
    if (sb[q] && cf[(int64_t)ocol[q] * b]) mx = fmax(mx, w[q]);
  int64_t J = -1;
  if (mx >= 0.0) {
    const double thr = mx * (1.0 - 1e-12);
    for (int64_t q = optr[I]; q < optr[I + 1] && J < 0; ++q)
      if (sb[q] && cf[(int64_t)ocol[q] * b] && w[q] >= thr) J = ocol[q];
  }
  for (int m = 0; m < b; ++m) pcol[I * b + m] = J >= 0 ? (int32_t)cidx[J * b + m] : -1;
}

template <int M, bool D2>
static void lair_launch(int64_t nc, const AhLevel& L, const uint8_t* strong, const int32_t* clist,
                        unsigned long long* nfall, hipStream_t st) {
  hipLaunchKernelGGL((k_lair<M, D2>), dim3((unsigned)nc), dim3(64), 0, st, nc, L.rowptr, L.col, L.val, strong, L.cf,
                     clist, L.Rptr, L.Rcol, L.Rval, nfall);
}

// lAIR restriction rows with local systems of capacity cap (8, 16, 32, 64)
// and distance-one or distance-two neighbourhoods.
static ah_status lair_dispatch(int cap, bool d2, int64_t nc, const AhLevel& L, const uint8_t* strong,
                               const int32_t* clist, unsigned long long* nfall, hipStream_t st) {
  if (nc == 0) return AH_OK;
  switch (cap) {
    case 8: d2 ? lair_launch<8, true>(nc, L, strong, clist, nfall, st) : lair_launch<8, false>(nc, L, strong, clist, nfall, st); break;
    case 16: d2 ? lair_launch<16, true>(nc, L, strong, clist, nfall, st) : lair_launch<16, false>(nc, L, strong, clist, nfall, st); break;
    case 32: d2 ? lair_launch<32, true>(nc, L, strong, clist, nfall, st) : lair_launch<32, false>(nc, L, strong, clist, nfall, st); break;
    default: d2 ? lair_launch<64, true>(nc, L, strong, clist, nfall, st) : lair_launch<64, false>(nc, L, strong, clist, nfall, st); break;
  }
  AH_LAUNCHED();
  return AH_OK;
}

// Block AIR lAIR rows, one wave per C block (capacity as lair_dispatch).
static ah_status lair_blk_dispatch(int cap, int64_t ncb, int b, const AhLevel& L, const uint8_t* strong,
                                   const int32_t* clist, unsigned long long* nfall, int* err, hipStream_t st) {
  if (ncb == 0) return AH_OK;
#define LB(M) hipLaunchKernelGGL((k_lair_blk<M>), dim3((unsigned)ncb), dim3(64), 0, st, ncb, b, L.rowptr, L.col, \
                                 L.val, strong, L.cf, clist, L.Rptr, L.Rcol, L.Rval, nfall, err)
  switch (cap) {
    case 8: LB(8); break;
    case 16: LB(16); break;
    case 32: LB(32); break;
    default: LB(64); break;
  }
#undef LB
  AH_LAUNCHED();
  return AH_OK;
}

template <int HS>
static ah_status rap_launch(int64_t nc, const AhLevel& L, int32_t* cnt, const int64_t* cptr, int32_t* ccol,
                            double* cval, bool numeric, hipStream_t st) {
  if (nc == 0) return AH_OK;
  if (numeric)
    hipLaunchKernelGGL((k_rap<HS, true>), dim3(nc), dim3(64), 0, st, nc, L.Rptr, L.Rcol, L.Rval, L.rowptr, L.col,
                       L.val, L.pcol, cnt, cptr, ccol, cval);
  else
    hipLaunchKernelGGL((k_rap<HS, false>), dim3(nc), dim3(64), 0, st, nc, L.Rptr, L.Rcol, L.Rval, L.rowptr, L.col,
                       L.val, L.pcol, cnt, cptr, ccol, cval);
  AH_LAUNCHED();
  return AH_OK;
}

static ah_status rap_dispatch(int hs, int64_t nc, const AhLevel& L, int32_t* cnt, const int64_t* cptr, int32_t* ccol,
                              double* cval, bool numeric, hipStream_t st) {
  switch (hs) {
    case 64: return rap_launch<64>(nc, L, cnt, cptr, ccol, cval, numeric, st);
    case 128: return rap_launch<128>(nc, L, cnt, cptr, ccol, cval, numeric, st);
    case 256: return rap_launch<256>(nc, L, cnt, cptr, ccol, cval, numeric, st);
    case 512: return rap_launch<512>(nc, L, cnt, cptr, ccol, cval, numeric, st);
    case 1024: return rap_launch<1024>(nc, L, cnt, cptr, ccol, cval, numeric, st);
    case 2048: return rap_launch<2048>(nc, L, cnt, cptr, ccol, cval, numeric, st);
    case 4096: return rap_launch<4096>(nc, L, cnt, cptr, ccol, cval, numeric, st);
  }
  set_error("R A P: row candidate count beyond the LDS hash capacity");
  return AH_EUNSUPPORTED;
}

// Undecided points of the rows 0 .. n-1 (or of list[0 .. n-1]): flag, then
// written at the flag's prefix sum.
__global__ void k_pmis_uflag(int64_t n, const int8_t* __restrict__ state, const int32_t* __restrict__ list,
                             const int64_t* __restrict__ nd, int32_t* __restrict__ flag) {
  const int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ii >= n) return;
  flag[ii] = (!nd || ii < *nd) && state[list ? list[ii] : ii] == 0 ? 1 : 0;
}

__global__ void k_pmis_ulist(int64_t n, const int32_t* __restrict__ list, const int32_t* __restrict__ flag,
                             const int64_t* __restrict__ pos, int32_t* __restrict__ out) {
  const int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ii < n && flag[ii]) out[pos[ii]] = list ? list[ii] : (int32_t)ii;
}

// Graphs from this many points on run their later PMIS rounds over a list
// of the undecided points (AH_PMIS_LIST_MIN overrides).
static int64_t pmis_list_min() {
  const char* e = std::getenv("AH_PMIS_LIST_MIN");
  return e ? (int64_t)std::atoll(e) : (int64_t)1 << 20;
}

// PMIS C/F splitting of the graph (n, rp, ci) over its strong entries:
// state[i] = 1 (C) or 2 (F).  key and nbmax hold n entries of scratch;
// flags[0..1] are the undecided flags of alternating rounds, flags[3] the
// single-workgroup round-overflow flag.
static ah_status pmis_split(int64_t n, const int64_t* rp, const int32_t* ci, const uint8_t* strong,
                            const int32_t* infl, int level, uint64_t* key, unsigned long long* nbmax, int8_t* state,
                            unsigned long long* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_pmis_init, g1(n), dim3(256), 0, st, n, infl, level, key, state);
  AH_HIP(hipGetLastError());
  AH_HIP(hipMemsetAsync(nbmax, 0, n * sizeof(unsigned long long), st));
  const char* wg_env = std::getenv("AH_PMIS_WG_MAX");   // at most PMIS_WG_MAX (its LDS size)
  const int64_t wg_max = wg_env ? std::min<int64_t>(std::atoll(wg_env), PMIS_WG_MAX) : (int64_t)PMIS_WG_MAX;
  if (n <= wg_max) {
    // small graph: every round in one workgroup, no host checks
    static std::once_flag once;
    std::call_once(once, [] {
      (void)hipFuncSetAttribute((const void*)k_pmis_wg, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(PMIS_WG_MAX * 17 + 64));
    });
    const unsigned lds = (unsigned)(((n * 17 + 7) / 8) * 8);
    hipLaunchKernelGGL(k_pmis_wg, dim3(1), dim3(1024), lds, st, (int)n, rp, ci, strong, key, state, flags + 3);
    AH_HIP(hipGetLastError());
    return AH_OK;
  }
  if (n < pmis_list_min()) {
    // rounds over all points (launch-latency bound: listing costs more)
    for (int round = 0;; ++round) {
      if (round > 10000) { set_error("air_setup: PMIS did not terminate"); return AH_EINVAL; }
      unsigned long long* left_d = flags + (round & 1);
      hipLaunchKernelGGL(k_pmis_nbmax, g1(n * PG), dim3(256), 0, st, n, rp, ci, strong, key, state, nbmax, nullptr,
                         nullptr);
      hipLaunchKernelGGL(k_pmis_select, g1(n), dim3(256), 0, st, n, key, nbmax, state, left_d, nullptr, nullptr);
      hipLaunchKernelGGL(k_pmis_fmark, grows(n), dim3(256), 0, st, n, rp, ci, strong, state, left_d, nullptr, nullptr);
      AH_HIP(hipGetLastError());
      // rounds run in pairs between host checks: a round after the last
      // undecided point is gone changes nothing and leaves its flag at 0
      if ((round & 1) == 0) continue;
      unsigned long long left = 0;
      AH_TRY(read_bytes(left_d, &left, sizeof(left), st));
      if (left == 0) return AH_OK;
    }
  }
  // large graphs: after each round the points still undecided are listed
  // (their count stays on the device; the grids are sized by the last count
  // read on the host, an upper bound), and the next round runs over that
  // list; the host reads the count every second round
  Arena tmp;
  tmp.stream = st;
  int32_t* lists[2] = {nullptr, nullptr};
  int32_t* flag = nullptr;
  int64_t* pos[2] = {nullptr, nullptr};
  ah_status rc = tmp.get(&lists[0], n);
  if (rc == AH_OK) rc = tmp.get(&lists[1], n);
  if (rc == AH_OK) rc = tmp.get(&flag, n);
  if (rc == AH_OK) rc = tmp.get(&pos[0], n + 1);
  if (rc == AH_OK) rc = tmp.get(&pos[1], n + 1);
  if (rc < 0) { tmp.release(); return rc; }
  const int32_t* list = nullptr;
  const int64_t* nd = nullptr;
  int64_t nl = n;   // host bound of the list length
  for (int round = 0;; ++round) {
    if (round > 10000) { tmp.release(); set_error("air_setup: PMIS did not terminate"); return AH_EINVAL; }
    unsigned long long* left_d = flags + (round & 1);
    hipLaunchKernelGGL(k_pmis_nbmax, g1(nl * PG), dim3(256), 0, st, nl, rp, ci, strong, key, state, nbmax, list, nd);
    hipLaunchKernelGGL(k_pmis_select, g1(nl), dim3(256), 0, st, nl, key, nbmax, state, left_d, list, nd);
    hipLaunchKernelGGL(k_pmis_fmark, grows(nl), dim3(256), 0, st, nl, rp, ci, strong, state, left_d, list, nd);
    int32_t* out = lists[round & 1];
    int64_t* p = pos[round & 1];
    hipLaunchKernelGGL(k_pmis_uflag, g1(nl), dim3(256), 0, st, nl, state, list, nd, flag);
    if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: PMIS round"); return AH_EHIP; }
    rc = scan_i32_to_i64(flag, p, nl, st, tmp);
    if (rc < 0) { tmp.release(); return rc; }
    hipLaunchKernelGGL(k_pmis_ulist, g1(nl), dim3(256), 0, st, nl, list, flag, p, out);
    if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: PMIS list"); return AH_EHIP; }
    list = out;
    nd = p + nl;
    if ((round & 1) == 0) continue;
    int64_t cnt = 0;
    rc = read_bytes(nd, &cnt, sizeof(cnt), st);
    if (rc < 0) { tmp.release(); return rc; }
    if (cnt == 0) { tmp.release(); return AH_OK; }
    nl = cnt;
  }
}

template <int HS, bool NUMERIC, int B>
static void rap_blk_launch(int64_t ncb, const AhLevel& L, const int32_t* clist, int32_t* cnt, const int64_t* cptr,
                           int32_t* ccol, double* cval, hipStream_t st) {
  hipLaunchKernelGGL((k_rap_blk<HS, NUMERIC, B>), dim3((unsigned)ncb), dim3(64), 0, st, ncb, L.Rptr, L.Rcol, L.Rval,
                     L.rowptr, L.col, L.val, L.pcol, clist, cnt, cptr, ccol, cval);
}

// Whether the block R A P kernels take blocks of b rows with hash size hs
// (the numeric pass keeps b sums per slot in LDS).
static bool rap_blk_fits(int b, int hs, bool numeric) {
  if (b != 2 && b != 3 && b != 6) return false;
  if (hs < 64 || hs > 4096) return false;
  return numeric ? hs * (12 + 8 * b) <= 65536 : true;
}

template <bool NUMERIC, int B>
static ah_status rap_blk_hs(int hs, int64_t ncb, const AhLevel& L, const int32_t* clist, int32_t* cnt,
                            const int64_t* cptr, int32_t* ccol, double* cval, hipStream_t st) {
  switch (hs) {
    case 64: rap_blk_launch<64, NUMERIC, B>(ncb, L, clist, cnt, cptr, ccol, cval, st); break;
    case 128: rap_blk_launch<128, NUMERIC, B>(ncb, L, clist, cnt, cptr, ccol, cval, st); break;
    case 256: rap_blk_launch<256, NUMERIC, B>(ncb, L, clist, cnt, cptr, ccol, cval, st); break;
    case 512: rap_blk_launch<512, NUMERIC, B>(ncb, L, clist, cnt, cptr, ccol, cval, st); break;
    case 1024: rap_blk_launch<1024, NUMERIC, B>(ncb, L, clist, cnt, cptr, ccol, cval, st); break;
    case 2048:
      if (NUMERIC) return AH_EUNSUPPORTED;
      rap_blk_launch<2048, false, B>(ncb, L, clist, cnt, cptr, ccol, cval, st);
      break;
    case 4096:
      if (NUMERIC) return AH_EUNSUPPORTED;
      rap_blk_launch<4096, false, B>(ncb, L, clist, cnt, cptr, ccol, cval, st);
      break;
    default: return AH_EUNSUPPORTED;
  }
  AH_LAUNCHED();
  return AH_OK;
}

static ah_status rap_blk_dispatch(int hs, int b, bool numeric, int64_t ncb, const AhLevel& L, const int32_t* clist,
                                  int32_t* cnt, const int64_t* cptr, int32_t* ccol, double* cval, hipStream_t st) {
  if (ncb == 0) return AH_OK;
  ah_status rc = AH_EUNSUPPORTED;
  if (b == 2) rc = numeric ? rap_blk_hs<true, 2>(hs, ncb, L, clist, cnt, cptr, ccol, cval, st)
                           : rap_blk_hs<false, 2>(hs, ncb, L, clist, cnt, cptr, ccol, cval, st);
  if (b == 3) rc = numeric ? rap_blk_hs<true, 3>(hs, ncb, L, clist, cnt, cptr, ccol, cval, st)
                           : rap_blk_hs<false, 3>(hs, ncb, L, clist, cnt, cptr, ccol, cval, st);
  if (b == 6) rc = numeric ? rap_blk_hs<true, 6>(hs, ncb, L, clist, cnt, cptr, ccol, cval, st)
                           : rap_blk_hs<false, 6>(hs, ncb, L, clist, cnt, cptr, ccol, cval, st);
  if (rc == AH_EUNSUPPORTED) set_error("block R A P: unsupported block size or hash size");
  return rc;
}

}  // namespace ah

using namespace ah;

// Ruge-Stueben first-pass coarsening on the host (the single-process form of
// the Falgout coarsening of Section 4; sequential by nature): from the
// strong entries of the CSR pattern, state[i] = 1 (C) or 2 (F).  The measure
// of an undecided point is the number of undecided points that depend on it
// strongly; points with measure 0 at the start are F; then the undecided
// point of largest measure (ties: smallest index) becomes C, the undecided
// points depending on it become F, each undecided point a new F point
// depends on gains one, each undecided point the new C point depends on
// loses one, and an undecided point whose measure reaches 0 becomes F.
static void rs_first_pass_host(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& col,
                               const std::vector<uint8_t>& strong, std::vector<int8_t>& state) {
  std::vector<int64_t> sp(n + 1, 0), tp(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
      if (strong[k]) { ++sp[i + 1]; ++tp[col[k] + 1]; }
  for (int64_t i = 0; i < n; ++i) { sp[i + 1] += sp[i]; tp[i + 1] += tp[i]; }
  std::vector<int32_t> sc(sp[n]), tc(tp[n]);
  {
    std::vector<int64_t> fs(sp.begin(), sp.end() - 1), ft(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
        if (strong[k]) { sc[fs[i]++] = col[k]; tc[ft[col[k]]++] = (int32_t)i; }
  }
  std::vector<int32_t> lam(n);
  state.assign(n, 0);
  std::priority_queue<std::pair<int32_t, int32_t>> heap;   // (measure, -index): largest, then smallest index
  for (int64_t i = 0; i < n; ++i) {
    lam[i] = (int32_t)(tp[i + 1] - tp[i]);
    if (lam[i] == 0) state[i] = 2;
    else heap.push({lam[i], -(int32_t)i});
  }
  while (!heap.empty()) {
    const auto top = heap.top();
    heap.pop();
    const int32_t i = -top.second;
    if (state[i] != 0 || top.first != lam[i]) continue;   // stale entry
    state[i] = 1;
    for (int64_t a = tp[i]; a < tp[i + 1]; ++a) {
      const int32_t j = tc[a];
      if (state[j] != 0) continue;
      state[j] = 2;
      for (int64_t b = sp[j]; b < sp[j + 1]; ++b) {
        const int32_t k = sc[b];
        if (state[k] == 0) heap.push({++lam[k], -k});
      }
    }
    for (int64_t b = sp[i]; b < sp[i + 1]; ++b) {
      const int32_t k = sc[b];
      if (state[k] != 0) continue;
      if (--lam[k] == 0) state[k] = 2;
      else heap.push({lam[k], -k});
    }
  }
}

ah_hier::~ah_hier() { arena.release(); }

// Level 0 under block AIR in sweep order: item k < nbF is the k-th F block
// (list[k B] / B of the F list), the rest the C blocks; each item's blocks
// (column indices and B x B values) copied to its range of the copy, 16
// lanes per item reading and writing contiguous runs.
__global__ void k_so_perm(int64_t n, const int32_t* __restrict__ list, int B, int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = list[k * B] / B;
}

__global__ void k_so_count(int64_t nbr, const int32_t* __restrict__ perm, const int64_t* __restrict__ optr,
                           int64_t* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nbr) cnt[k] = optr[perm[k] + 1] - optr[perm[k]];
}

__global__ void k_so_copy(int64_t nbr, int B, const int32_t* __restrict__ perm, const int64_t* __restrict__ optr,
                          const int32_t* __restrict__ ocol, const double* __restrict__ ov,
                          const int64_t* __restrict__ soptr, int32_t* __restrict__ socol, double* __restrict__ sov,
                          float* __restrict__ sov32) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = gid / 16;
  const int t = (int)(gid % 16);
  if (k >= nbr) return;
  const int64_t R = perm[k];
  const int64_t o = optr[R], p = soptr[k];
  const int64_t nb = optr[R + 1] - o;
  for (int64_t s = t; s < nb; s += 16) socol[p + s] = ocol[o + s];
  const int64_t bb = (int64_t)B * B;
  for (int64_t e = t; e < nb * bb; e += 16) {
    const double a = ov[o * bb + e];
    sov[p * bb + e] = a;
    if (sov32) sov32[p * bb + e] = (float)a;
  }
}

// The column encodings of the sweep-ordered copy for sweeps that read P e_c
// from e_c: with block one-point P, block J of P e_c is coarse block
// pcol[J B] / B of e_c (rows in order), or zero where pcol[J B] < 0; a C
// block's is its own coarse block.  An F column block is named by its F
// item (fpos: the sweeps keep the F blocks' values compact).  16 lanes per
// item.
__global__ void k_so_fpos(int64_t nbF, const int32_t* __restrict__ perm, int32_t* __restrict__ fpos) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nbF) fpos[perm[k]] = (int32_t)k;
}

__global__ void k_so_enc(int64_t nbr, int B, const int32_t* __restrict__ perm, const int64_t* __restrict__ soptr,
                         const int32_t* __restrict__ socol, const int32_t* __restrict__ pcol,
                         const int8_t* __restrict__ cf, const int32_t* __restrict__ fpos,
                         int32_t* __restrict__ socp, int32_t* __restrict__ soce, int32_t* __restrict__ soown,
                         int* __restrict__ bad) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = gid / 16;
  const int t = (int)(gid % 16);
  if (k >= nbr) return;
  for (int64_t o = soptr[k] + t; o < soptr[k + 1]; o += 16) {
    const int64_t J = socol[o];
    const int32_t pj = pcol[J * B];
    const int32_t cj = pj >= 0 ? pj / B : -1;
    // P must copy whole coarse blocks, and a C block must have its own
    if ((pj >= 0 && pj % B != 0) || (cf[J * B] && pj < 0)) *bad = 1;
    socp[o] = cj;
    soce[o] = cf[J * B] ? ~cj : fpos[J];
  }
  if (t == 0) {
    const int32_t pr = pcol[(int64_t)perm[k] * B];
    if (pr >= 0 && pr % B != 0) *bad = 1;
    soown[k] = pr >= 0 ? pr / B : -1;
  }
}

// Level 0 under scalar AIR in sweep order: item k of the concatenated F and
// C lists gets its row's values (nb B of them, row m of block row R at
// (optr[R] B + m nb) B) at off[k]; counts first, then 16 lanes per row.
__global__ void k_rso_count(int64_t n, const int32_t* __restrict__ items, int B, const int64_t* __restrict__ optr,
                            int64_t* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t R = items[k] / B;
  cnt[k] = (optr[R + 1] - optr[R]) * B;
}

__global__ void k_rso_copy(int64_t n, const int32_t* __restrict__ items, int B, const int64_t* __restrict__ optr,
                           const double* __restrict__ ov, const int64_t* __restrict__ off, double* __restrict__ sov,
                           float* __restrict__ sov32) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = gid / 16;
  const int t = (int)(gid % 16);
  if (k >= n) return;
  const int64_t i = items[k];
  const int64_t R = i / B;
  const int64_t len = (optr[R + 1] - optr[R]) * B;
  const double* __restrict__ v = ov + optr[R] * B * B + (i - R * B) * len;
  const int64_t p = off[k];
  for (int64_t e = t; e < len; e += 16) {
    const double a = v[e];
    sov[p + e] = a;
    if (sov32) sov32[p + e] = (float)a;
  }
}

static ah_status row_order_build(ah_hier* h, hipStream_t st) {
  AhLevel& L = h->lev[0];
  const int B = L.ob;
  const int64_t nF = L.n - L.nc;
  if (L.fblk || B < 2 || !L.oval || !L.flist || !L.clist || L.n == 0) return AH_OK;
  Arena& ar = h->arena;
  Arena tmp;
  tmp.stream = st;
  int64_t *cnt = nullptr, *off = nullptr;
  double* sov = nullptr;
  ah_status rc = tmp.get(&cnt, L.n);
  if (rc == AH_OK) rc = ar.get(&off, L.n + 1);
  if (rc == AH_OK) rc = ar.get(&sov, std::max<int64_t>(L.nov, 1));
  if (rc == AH_OK && h->prm.fp32_cycle) rc = ar.get(&L.soval32, std::max<int64_t>(L.nov, 1));
  if (rc < 0) { tmp.release(); return rc; }
  if (nF > 0) hipLaunchKernelGGL(k_rso_count, g1(nF), dim3(256), 0, st, nF, L.flist, B, L.optr, cnt);
  if (L.nc > 0) hipLaunchKernelGGL(k_rso_count, g1(L.nc), dim3(256), 0, st, L.nc, L.clist, B, L.optr, cnt + nF);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: row order count"); return AH_EHIP; }
  rc = scan_i64(cnt, off, L.n, st, tmp);
  if (rc < 0) { tmp.release(); return rc; }
  if (nF > 0)
    hipLaunchKernelGGL(k_rso_copy, g1(nF * 16), dim3(256), 0, st, nF, L.flist, B, L.optr, L.oval, off, sov, L.soval32);
  if (L.nc > 0)
    hipLaunchKernelGGL(k_rso_copy, g1(L.nc * 16), dim3(256), 0, st, L.nc, L.clist, B, L.optr, L.oval, off + nF, sov,
                       L.soval32);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: row order copy"); return AH_EHIP; }
  tmp.release();
  L.rsoff = off;
  L.soval = sov;
  return AH_OK;
}

static ah_status sweep_order_build(ah_hier* h, hipStream_t st) {
  AhLevel& L = h->lev[0];
  const int B = L.ob;
  if (!L.fblk || B < 2 || !L.oval || !L.flist || !L.clist) return AH_OK;
  const int64_t nbr = L.n / B, nbF = L.nF / B, nbC = L.nc / B;
  if (nbr * B != L.n || nbF * B != L.nF || nbC * B != L.nc || nbF + nbC != nbr) return AH_OK;
  Arena& ar = h->arena;
  Arena tmp;
  tmp.stream = st;
  int32_t *perm = nullptr, *socol = nullptr;
  int64_t *cnt = nullptr, *soptr = nullptr;
  double* sov = nullptr;
  const int64_t nblk = L.nov / ((int64_t)B * B);
  ah_status rc = tmp.get(&cnt, std::max<int64_t>(nbr, 1));
  if (rc == AH_OK) rc = ar.get(&perm, std::max<int64_t>(nbr, 1));
  if (rc == AH_OK) rc = ar.get(&soptr, nbr + 1);
  if (rc == AH_OK) rc = ar.get(&socol, std::max<int64_t>(nblk, 1));
  if (rc == AH_OK) rc = ar.get(&sov, std::max<int64_t>(L.nov, 1));
  if (rc == AH_OK && h->prm.fp32_cycle) rc = ar.get(&L.soval32, std::max<int64_t>(L.nov, 1));
  if (rc < 0) { tmp.release(); return rc; }
  if (nbF > 0) hipLaunchKernelGGL(k_so_perm, g1(nbF), dim3(256), 0, st, nbF, L.flist, B, perm);
  if (nbC > 0) hipLaunchKernelGGL(k_so_perm, g1(nbC), dim3(256), 0, st, nbC, L.clist, B, perm + nbF);
  hipLaunchKernelGGL(k_so_count, g1(nbr), dim3(256), 0, st, nbr, perm, L.optr, cnt);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: sweep order"); return AH_EHIP; }
  rc = scan_i64(cnt, soptr, nbr, st, tmp);
  if (rc < 0) { tmp.release(); return rc; }
  hipLaunchKernelGGL(k_so_copy, g1(nbr * 16), dim3(256), 0, st, nbr, B, perm, L.optr, L.ocol, L.oval, soptr, socol,
                     sov, L.soval32);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: sweep order copy"); return AH_EHIP; }
  tmp.release();
  L.sperm = perm;
  L.soptr = soptr;
  L.socol = socol;
  L.soval = sov;
  // the encodings for the sweeps without an interpolation pass
  if (L.pcol && L.cf && nbC > 0) {
    int32_t *socp = nullptr, *soce = nullptr, *soown = nullptr, *fpos = nullptr;
    int* d_bad = nullptr;
    Arena tmp2;
    tmp2.stream = st;
    rc = ar.get(&socp, std::max<int64_t>(nblk, 1));
    if (rc == AH_OK) rc = ar.get(&soce, std::max<int64_t>(nblk, 1));
    if (rc == AH_OK) rc = ar.get(&soown, std::max<int64_t>(nbr, 1));
    if (rc == AH_OK) rc = tmp2.get(&fpos, std::max<int64_t>(nbr, 1));
    if (rc == AH_OK) rc = tmp2.get(&d_bad, 1);
    if (rc < 0) { tmp2.release(); return rc; }
    if (hipMemsetAsync(d_bad, 0, sizeof(int), st) != hipSuccess) {
      tmp2.release();
      set_error("air_setup: sweep order encodings");
      return AH_EHIP;
    }
    if (nbF > 0) hipLaunchKernelGGL(k_so_fpos, g1(nbF), dim3(256), 0, st, nbF, perm, fpos);
    hipLaunchKernelGGL(k_so_enc, g1(nbr * 16), dim3(256), 0, st, nbr, B, perm, soptr, socol, L.pcol, L.cf, fpos,
                       socp, soce, soown, d_bad);
    int hbad = 0;
    rc = hipGetLastError() != hipSuccess ? AH_EHIP : read_bytes(d_bad, &hbad, sizeof(int), st);
    tmp2.release();
    if (rc != AH_OK) { set_error("air_setup: sweep order encodings"); return AH_EHIP; }
    // a P that does not copy whole coarse blocks keeps the interpolation pass
    if (hbad) return AH_OK;
    L.socp = socp;
    L.soce = soce;
    L.soown = soown;
  }
  return AH_OK;
}

// A CSR operator whose rows come in groups of B (block rows) read by the
// sweeps as full b x b blocks: block row I holds the distinct column blocks
// J (column / B) of its B rows; row m stores, per block s, the B values of
// columns J_s B + c at (m nb_I + s) B + c from the block row's value base.
// A block row is regular when its B rows have the same length, a multiple
// of B, and entry t of every row has column J B + t mod B with J the block
// of entry t - t mod B of the first row: then its CSR values are already in
// that layout, and the base is the CSR offset of its first row.  Other block
// rows get their blocks in a side array, in the order a merge of the rows
// meets them, zero where a row has no entry (every entry lands in exactly
// one slot, so a row's sum is its CSR sum); their base is stored as ~offset.
// One thread per block row.
template <int B>
__device__ __forceinline__ int32_t bfull_next(const int64_t* p, const int64_t* e, const int32_t* __restrict__ ci) {
  int32_t J = 0x7fffffff;
#pragma unroll
  for (int q = 0; q < B; ++q)
    if (p[q] < e[q]) J = min(J, ci[p[q]] / B);
  return J;
}

// Blocks of each block row (cnt), of which in the side array (acnt: all of
// an irregular block row's, none of a regular one's).  Eight lanes per
// block row check the pattern; the first lane counts an irregular row's
// blocks by the merge.
template <int B>
__global__ void k_bfull_count(int64_t nbr, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              int64_t* __restrict__ cnt, int64_t* __restrict__ acnt) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t I = gid / 8;
  const int g = (int)(gid % 8);
  if (I >= nbr) return;
  int64_t p[B], e[B];
#pragma unroll
  for (int q = 0; q < B; ++q) { p[q] = rp[I * B + q]; e[q] = rp[I * B + q + 1]; }
  const int64_t len = e[0] - p[0];
  bool reg = len % B == 0;
#pragma unroll
  for (int q = 1; q < B; ++q) reg = reg && e[q] - p[q] == len;
  if (reg)
    for (int64_t t = g; t < len; t += 8) {
      const int32_t J = ci[p[0] + t - t % B] / B;
#pragma unroll
      for (int q = 0; q < B; ++q) reg = reg && ci[p[q] + t] == J * B + (int32_t)(t % B);
    }
  int r = reg ? 1 : 0;
  for (int o = 4; o > 0; o >>= 1) r &= __shfl_xor(r, o, 8);
  if (g != 0) return;
  if (r) {
    cnt[I] = len / B;
    acnt[I] = 0;
    return;
  }
  int64_t c = 0;
  for (int32_t J = bfull_next<B>(p, e, ci); J != 0x7fffffff; J = bfull_next<B>(p, e, ci)) {
    ++c;
#pragma unroll
    for (int q = 0; q < B; ++q)
      while (p[q] < e[q] && ci[p[q]] / B == J) ++p[q];
  }
  cnt[I] = c;
  acnt[I] = c;
}

// Block columns and value bases of every block row; the side-array blocks
// of the irregular ones.
template <int B>
__global__ void k_bfull_fill(int64_t nbr, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const double* __restrict__ v, const int64_t* __restrict__ bptr,
                             const int64_t* __restrict__ aptr, int32_t* __restrict__ bcol,
                             int64_t* __restrict__ voff, double* __restrict__ aux) {
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nbr) return;
  int64_t p[B], e[B];
#pragma unroll
  for (int q = 0; q < B; ++q) { p[q] = rp[I * B + q]; e[q] = rp[I * B + q + 1]; }
  const int64_t o0 = bptr[I];
  const int64_t nb = bptr[I + 1] - o0;
  const int64_t a0 = aptr[I];
  if (aptr[I + 1] == a0) {     // regular (or empty): values in place
    for (int64_t s = 0; s < nb; ++s) bcol[o0 + s] = ci[p[0] + s * B] / B;
    voff[I] = p[0];
    return;
  }
  voff[I] = ~(a0 * (B * B));
  double* __restrict__ vb = aux + a0 * (B * B);
  int64_t s = 0;
  for (int32_t J = bfull_next<B>(p, e, ci); J != 0x7fffffff && s < nb; J = bfull_next<B>(p, e, ci), ++s) {
    bcol[o0 + s] = J;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      double* __restrict__ w = vb + (q * nb + s) * B;
#pragma unroll
      for (int c = 0; c < B; ++c) w[c] = 0.0;
      while (p[q] < e[q] && ci[p[q]] / B == J) {
        w[ci[p[q]] - J * B] = v[p[q]];
        ++p[q];
      }
    }
  }
}

// The rows of a level read by full blocks, copied in sweep order: item k of
// the concatenated F and C lists gets its row's values (nb B of them) at
// off[k]; cnt_k first, then the copy with 16 lanes per row, which also
// writes the item's record (value offset, first block column, blocks).
__global__ void k_bso_count(int64_t n, const int32_t* __restrict__ items, int B, const int64_t* __restrict__ bptr,
                            int64_t* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t R = items[k] / B;
  cnt[k] = (bptr[R + 1] - bptr[R]) * B;
}

__global__ void k_bso_copy(int64_t n, const int32_t* __restrict__ items, int B, const int64_t* __restrict__ bptr,
                           const int64_t* __restrict__ voff, const double* __restrict__ av,
                           const double* __restrict__ ax, const int64_t* __restrict__ off, double* __restrict__ sov,
                           float* __restrict__ sov32, AhRowRec* __restrict__ rec) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = gid / 16;
  const int t = (int)(gid % 16);
  if (k >= n) return;
  const int64_t i = items[k];
  const int64_t R = i / B;
  const int64_t nb = bptr[R + 1] - bptr[R];
  const int64_t len = nb * B;
  const int64_t vo = voff[R];
  const double* __restrict__ v = (vo >= 0 ? av + vo : ax + ~vo) + (i - R * B) * len;
  const int64_t p = off[k];
  if (t == 0) {
    AhRowRec r;
    r.voff = p;
    r.o0 = (int32_t)bptr[R];
    r.nb = (int32_t)nb;
    rec[k] = r;
  }
  for (int64_t e = t; e < len; e += 16) {
    const double a = v[e];
    sov[p + e] = a;
    if (sov32) sov32[p + e] = (float)a;
  }
}

// The restriction of a block AIR level, R = [Z I], by coarse blocks: the B
// rows of coarse block k (fine block i0 / B, i0 = clist[k B]) hold the same
// neighbourhood columns, whole F blocks in increasing order, and their own
// column i0 + q with the value 1.  k_rz_count counts the neighbourhood
// blocks and flags (*bad) a block row that is not of that form; k_rz_fill
// writes Z's blocks (row q of block s at (zptr[k] B + q nb + s) B) and the
// column blocks.  One thread per coarse block.
__global__ void k_rz_count(int64_t ncb, int B, const int64_t* __restrict__ Rptr, int64_t* __restrict__ cnt,
                           int* __restrict__ bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncb) return;
  const int64_t len = Rptr[k * B + 1] - Rptr[k * B];
  bool ok = len >= 1 && (len - 1) % B == 0;
  for (int q = 1; q < B; ++q) ok = ok && Rptr[k * B + q + 1] - Rptr[k * B + q] == len;
  cnt[k] = ok ? (len - 1) / B : 0;
  if (!ok) atomicOr(bad, 1);
}

__global__ void k_rz_fill(int64_t ncb, int B, const int64_t* __restrict__ Rptr, const int32_t* __restrict__ Rcol,
                          const double* __restrict__ Rval, const int32_t* __restrict__ clist,
                          const int64_t* __restrict__ zptr, int32_t* __restrict__ zcol, double* __restrict__ zval,
                          int* __restrict__ bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncb) return;
  const int64_t i0 = clist[k * B];
  const int64_t z0 = zptr[k];
  const int64_t nb = zptr[k + 1] - z0;
  bool ok = i0 % B == 0;
  for (int q = 0; q < B && ok; ++q) {
    ok = ok && clist[k * B + q] == i0 + q;
    const int64_t base = Rptr[k * B + q], len = Rptr[k * B + q + 1] - base;
    int64_t pos = 0;
    bool own = false;
    for (int64_t t = 0; t < len && ok; ++t) {
      const int32_t c = Rcol[base + t];
      if (c >= i0 && c < i0 + B) {
        ok = !own && c == i0 + q && Rval[base + t] == 1.0;
        own = true;
        continue;
      }
      const int64_t sb = pos / B;
      const int cc = (int)(pos % B);
      if (sb >= nb || c % B != cc) { ok = false; break; }
      if (q == 0 && cc == 0) zcol[z0 + sb] = c / B;
      else ok = ok && zcol[z0 + sb] == c / B;
      zval[z0 * B * B + (q * nb + sb) * B + cc] = Rval[base + t];
      ++pos;
    }
    ok = ok && own && pos == nb * B;
  }
  if (!ok) atomicOr(bad, 1);
}

// Z of block AIR level 0 by coarse blocks for the restriction; left unbuilt
// where a block row is not of the form (the CSR R is used then).
static ah_status rz_build(ah_hier* h, hipStream_t st) {
  AhLevel& L = h->lev[0];
  const int B = L.ob;
  if (!L.fblk || B < 2 || !L.clist || L.nc == 0 || L.nc % B) return AH_OK;
  const int64_t ncb = L.nc / B;
  Arena& ar = h->arena;
  Arena tmp;
  tmp.stream = st;
  int64_t *cnt = nullptr, *zptr = nullptr;
  int* bad = nullptr;
  ah_status rc = tmp.get(&cnt, ncb);
  if (rc == AH_OK) rc = tmp.get(&bad, 1);
  if (rc == AH_OK) rc = ar.get(&zptr, ncb + 1);
  if (rc < 0) { tmp.release(); return rc; }
  if (hipMemsetAsync(bad, 0, sizeof(int), st) != hipSuccess) { tmp.release(); set_error("air_setup: R blocks"); return AH_EHIP; }
  hipLaunchKernelGGL(k_rz_count, g1(ncb), dim3(256), 0, st, ncb, B, L.Rptr, cnt, bad);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: R blocks count"); return AH_EHIP; }
  rc = scan_i64(cnt, zptr, ncb, st, tmp);
  if (rc < 0) { tmp.release(); return rc; }
  double* pin = pinned_scratch(2);
  if (!pin) { tmp.release(); set_error("pinned host allocation failed"); return AH_ENOMEM; }
  int hbad = 0;
  int64_t nblk = 0;
  if (hipMemcpyAsync(pin, zptr + ncb, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(reinterpret_cast<char*>(pin) + 8, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    tmp.release();
    set_error("air_setup: R blocks readback");
    return AH_EHIP;
  }
  std::memcpy(&nblk, pin, sizeof(nblk));
  std::memcpy(&hbad, reinterpret_cast<char*>(pin) + 8, sizeof(hbad));
  if (hbad) { tmp.release(); return AH_OK; }
  const int64_t nv = nblk * B * B;
  int32_t* zcol = nullptr;
  double* zval = nullptr;
  rc = ar.get(&zcol, std::max<int64_t>(nblk, 1));
  if (rc == AH_OK) rc = ar.get(&zval, std::max<int64_t>(nv, 1));
  if (rc < 0) { tmp.release(); return rc; }
  hipLaunchKernelGGL(k_rz_fill, g1(ncb), dim3(256), 0, st, ncb, B, L.Rptr, L.Rcol, L.Rval, L.clist, zptr, zcol, zval,
                     bad);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(reinterpret_cast<char*>(pin) + 8, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    tmp.release();
    set_error("air_setup: R blocks fill");
    return AH_EHIP;
  }
  std::memcpy(&hbad, reinterpret_cast<char*>(pin) + 8, sizeof(hbad));
  tmp.release();
  if (hbad) return AH_OK;
  if (h->prm.fp32_cycle) {
    AH_TRY(ar.get(&L.rzval32, std::max<int64_t>(nv, 1)));
    if (nv > 0) hipLaunchKernelGGL(k_cast32, g1(nv), dim3(256), 0, st, nv, zval, L.rzval32);
    AH_LAUNCHED();
  }
  L.rzptr = zptr;
  L.rzcol = zcol;
  L.rzval = zval;
  L.nrz = nv;
  return AH_OK;
}

// The rows of a CSR level copied in sweep order: item k of the concatenated
// F and C lists gets its row's entries at off[k]; counts first, then the
// copy with 16 lanes per row.
__global__ void k_cso_count(int64_t n, const int32_t* __restrict__ items, const int64_t* __restrict__ rp,
                            int64_t* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) cnt[k] = rp[items[k] + 1] - rp[items[k]];
}

__global__ void k_cso_copy(int64_t n, const int32_t* __restrict__ items, const int64_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const double* __restrict__ v,
                           const int64_t* __restrict__ off, int32_t* __restrict__ oc, double* __restrict__ ov,
                           float* __restrict__ ov32) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = gid / 16;
  const int t = (int)(gid % 16);
  if (k >= n) return;
  const int64_t i = items[k];
  const int64_t s0 = rp[i], len = rp[i + 1] - s0, p = off[k];
  for (int64_t e = t; e < len; e += 16) {
    oc[p + e] = ci[s0 + e];
    const double a = v[s0 + e];
    ov[p + e] = a;
    if (ov32) ov32[p + e] = (float)a;
  }
}

// The sweep-ordered copy of CSR level l (FP64 and, for the FP32 cycle, FP32).
static ah_status csr_order_build(ah_hier* h, int l, hipStream_t st) {
  AhLevel& L = h->lev[l];
  const int64_t nF = L.n - L.nc;
  if (!L.flist || !L.clist || L.n == 0) return AH_OK;
  Arena& ar = h->arena;
  Arena tmp;
  tmp.stream = st;
  int64_t *cnt = nullptr, *off = nullptr;
  int32_t* oc = nullptr;
  double* ov = nullptr;
  ah_status rc = tmp.get(&cnt, L.n);
  if (rc == AH_OK) rc = ar.get(&off, L.n + 1);
  if (rc == AH_OK) rc = ar.get(&oc, std::max<int64_t>(L.nnz, 1));
  if (rc == AH_OK) rc = ar.get(&ov, std::max<int64_t>(L.nnz, 1));
  if (rc == AH_OK && h->prm.fp32_cycle) rc = ar.get(&L.coval32, std::max<int64_t>(L.nnz, 1));
  if (rc < 0) { tmp.release(); return rc; }
  if (nF > 0) hipLaunchKernelGGL(k_cso_count, g1(nF), dim3(256), 0, st, nF, L.flist, L.rowptr, cnt);
  if (L.nc > 0) hipLaunchKernelGGL(k_cso_count, g1(L.nc), dim3(256), 0, st, L.nc, L.clist, L.rowptr, cnt + nF);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: level order count"); return AH_EHIP; }
  rc = scan_i64(cnt, off, L.n, st, tmp);
  if (rc < 0) { tmp.release(); return rc; }
  if (nF > 0)
    hipLaunchKernelGGL(k_cso_copy, g1(nF * 16), dim3(256), 0, st, nF, L.flist, L.rowptr, L.col, L.val, off, oc, ov,
                       L.coval32);
  if (L.nc > 0)
    hipLaunchKernelGGL(k_cso_copy, g1(L.nc * 16), dim3(256), 0, st, L.nc, L.clist, L.rowptr, L.col, L.val, off + nF,
                       oc, ov, L.coval32);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: level order copy"); return AH_EHIP; }
  tmp.release();
  L.coptr = off;
  L.cocol = oc;
  L.coval = ov;
  return AH_OK;
}

// The full-block view of level l (block size B) for its F and C sweeps, if
// it stores at most 1.25 times the CSR entries; otherwise the level keeps
// the CSR sweeps.  Also the F rows' stored values (sweep byte counts) and
// the FP32 side array for the FP32 cycle.
// The values of the F rows, then of the C rows, of a level read by full
// blocks, in that order (FP64 and, for the FP32 cycle, FP32).
static ah_status block_view_order(ah_hier* h, int l, hipStream_t st) {
  AhLevel& L = h->lev[l];
  const int B = L.bb;
  const int64_t nF = L.n - L.nc;
  if (!L.flist || !L.clist) return AH_OK;
  Arena& ar = h->arena;
  Arena tmp;
  tmp.stream = st;
  // the records hold the first block column of a row as int32
  if (L.nbv / ((int64_t)B * B) >= (int64_t)INT32_MAX) return AH_OK;
  int64_t *cnt = nullptr, *off = nullptr;
  AhRowRec* rec = nullptr;
  double* sov = nullptr;
  ah_status rc = tmp.get(&cnt, std::max<int64_t>(L.n, 1));
  if (rc == AH_OK) rc = tmp.get(&off, L.n + 1);
  if (rc == AH_OK) rc = ar.get(&rec, std::max<int64_t>(L.n, 1));
  if (rc == AH_OK) rc = ar.get(&sov, std::max<int64_t>(L.nbv, 1));
  if (rc == AH_OK && h->prm.fp32_cycle) rc = ar.get(&L.soval32, std::max<int64_t>(L.nbv, 1));
  if (rc < 0) { tmp.release(); return rc; }
  if (nF > 0) hipLaunchKernelGGL(k_bso_count, g1(nF), dim3(256), 0, st, nF, L.flist, B, L.bptr, cnt);
  if (L.nc > 0) hipLaunchKernelGGL(k_bso_count, g1(L.nc), dim3(256), 0, st, L.nc, L.clist, B, L.bptr, cnt + nF);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: level order count"); return AH_EHIP; }
  rc = scan_i64(cnt, off, L.n, st, tmp);
  if (rc < 0) { tmp.release(); return rc; }
  if (nF > 0)
    hipLaunchKernelGGL(k_bso_copy, g1(nF * 16), dim3(256), 0, st, nF, L.flist, B, L.bptr, L.bvoff, L.val, L.baux, off,
                       sov, L.soval32, rec);
  if (L.nc > 0)
    hipLaunchKernelGGL(k_bso_copy, g1(L.nc * 16), dim3(256), 0, st, L.nc, L.clist, B, L.bptr, L.bvoff, L.val, L.baux,
                       off + nF, sov, L.soval32, rec + nF);
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: level order copy"); return AH_EHIP; }
  tmp.release();
  L.bsrec = rec;
  L.soval = sov;
  return AH_OK;
}

static ah_status block_view_build(ah_hier* h, int l, int B, hipStream_t st, bool so) {
  AhLevel& L = h->lev[l];
  const int64_t nbr = L.n / B;
  if (nbr == 0 || nbr * B != L.n || !L.flist || (B != 2 && B != 3 && B != 6)) return AH_OK;
  Arena tmp;
  tmp.stream = st;
  int64_t *cnt = nullptr, *acnt = nullptr, *bptr = nullptr, *aptr = nullptr, *voff = nullptr;
  unsigned long long* d_cnt = nullptr;
  ah_status rc = tmp.get(&cnt, nbr);
  if (rc == AH_OK) rc = tmp.get(&acnt, nbr);
  if (rc == AH_OK) rc = tmp.get(&aptr, nbr + 1);
  if (rc == AH_OK) rc = tmp.get(&d_cnt, 1);
  if (rc == AH_OK) rc = h->arena.get(&bptr, nbr + 1);
  if (rc == AH_OK) rc = h->arena.get(&voff, nbr);
  if (rc < 0) { tmp.release(); return rc; }
  switch (B) {
    case 2: hipLaunchKernelGGL(k_bfull_count<2>, g1(nbr * 8), dim3(256), 0, st, nbr, L.rowptr, L.col, cnt, acnt); break;
    case 3: hipLaunchKernelGGL(k_bfull_count<3>, g1(nbr * 8), dim3(256), 0, st, nbr, L.rowptr, L.col, cnt, acnt); break;
    default: hipLaunchKernelGGL(k_bfull_count<6>, g1(nbr * 8), dim3(256), 0, st, nbr, L.rowptr, L.col, cnt, acnt); break;
  }
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: block view count"); return AH_EHIP; }
  rc = scan_i64(cnt, bptr, nbr, st, tmp);
  if (rc == AH_OK) rc = scan_i64(acnt, aptr, nbr, st, tmp);
  if (rc < 0) { tmp.release(); return rc; }
  double* pin = pinned_scratch(2);
  if (!pin) { tmp.release(); set_error("pinned host allocation failed"); return AH_ENOMEM; }
  if (hipMemcpyAsync(pin, bptr + nbr, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(pin + 1, aptr + nbr, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    tmp.release();
    set_error("air_setup: block view count readback");
    return AH_EHIP;
  }
  int64_t tot[2] = {0, 0};
  std::memcpy(tot, pin, sizeof(tot));
  const int64_t nv = tot[0] * B * B, na = tot[1] * B * B;
  if ((double)nv > 1.25 * (double)L.nnz) { tmp.release(); return AH_OK; }
  int32_t* bcol = nullptr;
  double* aux = nullptr;
  rc = h->arena.get(&bcol, std::max<int64_t>(tot[0], 1));
  if (rc == AH_OK) rc = h->arena.get(&aux, std::max<int64_t>(na, 1));
  if (rc < 0) { tmp.release(); return rc; }
  switch (B) {
    case 2: hipLaunchKernelGGL(k_bfull_fill<2>, g1(nbr), dim3(256), 0, st, nbr, L.rowptr, L.col, L.val, bptr, aptr, bcol, voff, aux); break;
    case 3: hipLaunchKernelGGL(k_bfull_fill<3>, g1(nbr), dim3(256), 0, st, nbr, L.rowptr, L.col, L.val, bptr, aptr, bcol, voff, aux); break;
    default: hipLaunchKernelGGL(k_bfull_fill<6>, g1(nbr), dim3(256), 0, st, nbr, L.rowptr, L.col, L.val, bptr, aptr, bcol, voff, aux); break;
  }
  if (hipGetLastError() != hipSuccess) { tmp.release(); set_error("air_setup: block view fill"); return AH_EHIP; }
  if (h->prm.fp32_cycle) {
    rc = h->arena.get(&L.baux32, std::max<int64_t>(na, 1));
    if (rc < 0) { tmp.release(); return rc; }
    if (na > 0) hipLaunchKernelGGL(k_cast32, g1(na), dim3(256), 0, st, na, aux, L.baux32);
  }
  const int64_t nF = L.n - L.nc;
  if (hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long), st) != hipSuccess) {
    tmp.release();
    set_error("air_setup: block view counts");
    return AH_EHIP;
  }
  if (nF > 0) hipLaunchKernelGGL(k_list_vals, grows(nF), dim3(256), 0, st, nF, L.flist, bptr, B, d_cnt);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(pin, d_cnt, sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    tmp.release();
    set_error("air_setup: block view readback");
    return AH_EHIP;
  }
  tmp.release();
  unsigned long long nvF = 0;
  std::memcpy(&nvF, pin, sizeof(nvF));
  L.bb = B;
  if (const char* e = std::getenv("AH_L1LP")) {
    const int v = std::atoi(e);
    L.blp = (v == 2 || v == 4 || v == 8) ? v : 0;
  }
  L.nbv = nv;
  L.nbvF = (int64_t)nvF;
  L.nbaux = na;
  L.bptr = bptr;
  L.bcol = bcol;
  L.bvoff = voff;
  L.baux = aux;
  return so ? block_view_order(h, l, st) : AH_OK;
}

extern "C" void ah_air_defaults(ah_air_params* p) {
  if (!p) return;
  p->theta = 0.25;
  p->max_coarse = 64;
  p->max_levels = 25;
  p->relax = 0;
  p->omega = 1.0;
  p->stall = 0.9;
  p->fp32_cycle = 0;
  p->adjoint = 0;
  p->lair_distance = 1;
  p->theta_r = 0.0;
  p->order_ratio = 1.5;
  p->coarsening = 0;
  p->block_air = 0;
}

extern "C" ah_status air_setup(const ah_system* s, const ah_air_params* prm_in, void* stream, ah_hier** out,
                               ah_setup_info* info) {
  if (!s || !out) { set_error("air_setup: null argument"); return AH_EINVAL; }
  *out = nullptr;
  ah_air_params prm;
  if (prm_in) prm = *prm_in; else ah_air_defaults(&prm);
  if (prm.lair_distance == 0) prm.lair_distance = 1;
  if (prm.order_ratio == 0.0) prm.order_ratio = 1.5;
  if (prm.max_levels < 1 || prm.max_levels > 32 || !(prm.theta >= 0.0) || prm.max_coarse < 1 ||
      (prm.lair_distance != 1 && prm.lair_distance != 2) || !(prm.theta_r <= 1.0) || prm.relax < 0 ||
      prm.relax > 3 || !(prm.order_ratio >= 1.0 && prm.order_ratio < 1e300) || prm.coarsening < 0 ||
      prm.coarsening > 1 || prm.block_air < 0 || prm.block_air > 1) {
    set_error("air_setup: invalid parameters");
    return AH_EINVAL;
  }
  if (prm.block_air && (!s->d_odv || s->b < 2 || prm.lair_distance != 1 || prm.coarsening != 0)) {
    set_error("air_setup: block AIR needs a scaled system with facet blocks, lAIR distance one and PMIS");
    return AH_EINVAL;
  }
  hipStream_t st = as_stream(stream);
  auto t0 = std::chrono::steady_clock::now();
  ah_hier* h = new ah_hier();
  h->sys = s;
  h->prm = prm;
  h->arena.stream = st;
  Arena& ar = h->arena;
  Arena tmp;
  tmp.stream = st;
  ah_status rc = AH_OK;
#define CK(x) do { rc = (x); if (rc < 0) { tmp.release(); delete h; return rc; } } while (0)
#define CKH(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { set_error("air_setup: %s", hipGetErrorString(e_)); tmp.release(); delete h; return AH_EHIP; } } while (0)
  unsigned long long* d_ull = nullptr;   // [0..1] undecided counts (alternating rounds), [2] lAIR fallbacks,
                                         // [3] single-workgroup PMIS round overflow
  int* d_int = nullptr;                  // [0] max |N_i|, [1] max candidates, [2] max C-row length (then error flags), [3] max A_c row
  unsigned long long* d_fst = nullptr;   // per level: F rows, F-row entries
  CK(ar.get(&d_ull, 4));
  CK(ar.get(&d_int, 4));
  CK(ar.get(&d_fst, 66));   // [2 l], [2 l + 1] per level; [64] level-0 F values in the facet-block layout
  CKH(hipMemsetAsync(d_fst, 0, 66 * sizeof(unsigned long long), st));
  CKH(hipMemsetAsync(d_ull, 0, 4 * sizeof(unsigned long long), st));
  CKH(hipMemsetAsync(d_int, 0, 4 * sizeof(int), st));
  // level 0 = the scaled system (shared, not copied)
  AhLevel L0;
  L0.n = s->n;
  L0.nnz = s->nnz;
  L0.rowptr = s->d_rowptr;
  L0.col = s->d_col;
  L0.val = s->d_val;
  if (s->d_odv) {
    L0.ob = s->b;
    L0.nov = (int64_t)s->mesh->odb_col.size() * s->b * s->b;
    L0.optr = s->mesh->d_odb_ptr;
    L0.ocol = s->mesh->d_odb_col;
    L0.oval = s->d_odv;
  }
  h->lev.push_back(L0);
  // the tail never holds level 0 when it has more rows than this
  int64_t tail_max = 4096;
  if (const char* e = std::getenv("AH_TAIL_MAX")) tail_max = std::atoll(e);
  // adjoint: level 0 of a scaled system gets its transpose in the
  // facet-block layout, and no CSR transpose unless the ordered sweeps or the
  // tail need it
  bool at0_csr = true;
  for (int l = 0;; ++l) {
    AhLevel& L = h->lev[l];
    const int64_t n = L.n;
    CK(ar.get(&L.diag, n));
    if (prm.fp32_cycle) {
      CK(ar.get(&L.diag32, n));
      CK(ar.get(&L.val32, L.nnz));
      hipLaunchKernelGGL(k_cast32, g1(L.nnz), dim3(256), 0, st, L.nnz, L.val, L.val32);
      CKH(hipGetLastError());
      if (L.ob) {
        CK(ar.get(&L.oval32, L.nov));
        hipLaunchKernelGGL(k_cast32, g1(L.nov), dim3(256), 0, st, L.nov, L.oval, L.oval32);
        CKH(hipGetLastError());
      }
    }
    hipLaunchKernelGGL(k_diag, g1(n * PG), dim3(256), 0, st, n, L.rowptr, L.col, L.val, L.diag, L.diag32);
    CKH(hipGetLastError());
    CK(ar.get(&L.b, n)); CK(ar.get(&L.x, n)); CK(ar.get(&L.y, n)); CK(ar.get(&L.e, n));
    if (prm.fp32_cycle) {
      CK(ar.get(&L.b32, n)); CK(ar.get(&L.x32, n)); CK(ar.get(&L.y32, n)); CK(ar.get(&L.e32, n));
    }
    if (n <= prm.max_coarse || l == prm.max_levels - 1) break;
    // block AIR on level 0: strength and PMIS on the facet-block graph, the
    // scalar strong mask (restriction threshold) and the states expanded
    // to the rows of each block; P follows after the scalar pass below
    const bool blk = prm.block_air && l == 0;
    const int64_t nbr = blk ? n / L.ob : 0;
    double* bw = nullptr;
    uint8_t* sb = nullptr;
    uint8_t* strong = nullptr;
    int8_t* state = nullptr;
    CK(tmp.get(&strong, L.nnz));
    CK(tmp.get(&state, n));
    if (blk) {
      const int64_t nslot = (int64_t)s->mesh->odb_col.size();
      int32_t* infl = nullptr;
      uint64_t* key = nullptr;
      unsigned long long* nbmax = nullptr;
      int8_t* sbstate = nullptr;
      CK(tmp.get(&bw, nslot));
      CK(tmp.get(&sb, nslot));
      CK(tmp.get(&infl, nbr));
      CK(tmp.get(&key, nbr));
      CK(tmp.get(&nbmax, nbr));
      CK(tmp.get(&sbstate, nbr));
      hipLaunchKernelGGL(k_block_weights, g1(nbr * SG), dim3(256), 0, st, nbr, (int)L.ob, L.optr, L.oval, bw);
      CKH(hipMemsetAsync(infl, 0, nbr * sizeof(int32_t), st));
      hipLaunchKernelGGL(k_strength, g1(nbr * SG), dim3(256), 0, st, nbr, L.optr, L.ocol, bw, prm.theta, sb, infl);
      CKH(hipGetLastError());
      CK(pmis_split(nbr, L.optr, L.ocol, sb, infl, l, key, nbmax, sbstate, d_ull, st));
      hipLaunchKernelGGL(k_block_expand, g1(n), dim3(256), 0, st, n, (int)L.ob, sbstate, state);
      uint8_t* sbr = sb;
      if (prm.theta_r > 0.0 && prm.theta_r != prm.theta) {
        CK(tmp.get(&sbr, nslot));
        CKH(hipMemsetAsync(infl, 0, nbr * sizeof(int32_t), st));
        hipLaunchKernelGGL(k_strength, g1(nbr * SG), dim3(256), 0, st, nbr, L.optr, L.ocol, bw, prm.theta_r, sbr,
                           infl);
      }
      hipLaunchKernelGGL(k_block_mask, g1(n * PG), dim3(256), 0, st, n, (int)L.ob, L.rowptr, L.col, L.optr, L.ocol,
                         sbr, strong);
      CKH(hipGetLastError());
    } else {
    // strength
    int32_t* infl = nullptr;
    CK(tmp.get(&infl, n));
    CKH(hipMemsetAsync(infl, 0, n * sizeof(int32_t), st));
    hipLaunchKernelGGL(k_strength, g1(n * SG), dim3(256), 0, st, n, L.rowptr, L.col, L.val, prm.theta, strong, infl);
    CKH(hipGetLastError());
    // PMIS
    uint64_t* key = nullptr;
    unsigned long long* nbmax = nullptr;
    CK(tmp.get(&key, n));
    CK(tmp.get(&nbmax, n));
    if (prm.coarsening == 1) {
      // Ruge-Stueben first pass on the host from the strong pattern
      std::vector<int64_t> hrp(n + 1);
      std::vector<int32_t> hcol(L.nnz);
      std::vector<uint8_t> hst(L.nnz);
      std::vector<int8_t> hstate;
      CKH(hipMemcpyAsync(hrp.data(), L.rowptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
      CKH(hipMemcpyAsync(hcol.data(), L.col, L.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      CKH(hipMemcpyAsync(hst.data(), strong, L.nnz, hipMemcpyDeviceToHost, st));
      CKH(hipStreamSynchronize(st));
      rs_first_pass_host(n, hrp, hcol, hst, hstate);
      CKH(hipMemcpyAsync(state, hstate.data(), n, hipMemcpyHostToDevice, st));
      CKH(hipStreamSynchronize(st));
    } else {
      CK(pmis_split(n, L.rowptr, L.col, strong, infl, l, key, nbmax, state, d_ull, st));
    }
    }
    // coarse numbering
    int32_t* isc = nullptr;
    int64_t* cidx = nullptr;
    CK(ar.get(&L.cf, n));
    CK(tmp.get(&isc, n));
    CK(tmp.get(&cidx, n + 1));
    hipLaunchKernelGGL(k_cf_flags, g1(n), dim3(256), 0, st, n, state, L.cf, isc);
    CKH(hipGetLastError());
    CK(scan_i32_to_i64(isc, cidx, n, st, tmp));
    const bool d2 = prm.lair_distance == 2;
    int64_t nc = 0;
    // distance one: the point lists and R's row counts are sized for n, and
    // the C-point count is read back together with R's size (one host sync
    // per level instead of two); distance two needs it for its launches
    if (d2) {
      CK(read_i64(cidx + n, &nc, st));
      if (nc == 0 || (double)nc > prm.stall * (double)n) break;
    }
    const int64_t ncap = d2 ? nc : n;
    // one-point P, lAIR row lengths, R A P candidate bound, F-row statistics
    int32_t *rcnt = nullptr, *clist = nullptr;
    CK(ar.get(&L.pcol, n));
    CK(tmp.get(&rcnt, ncap + 1));
    CK(ar.get(&clist, ncap));
    CK(ar.get(&L.flist, n - (d2 ? nc : 0)));
    if (!d2) CKH(hipMemsetAsync(rcnt, 0, (n + 1) * sizeof(int32_t), st));
    CKH(hipMemsetAsync(d_int, 0, 4 * sizeof(int), st));
    // strength of the restriction neighbourhoods (theta_r; the same mask
    // when it equals theta)
    uint8_t* strong_r = strong;
    if (!blk && prm.theta_r > 0.0 && prm.theta_r != prm.theta) {
      int32_t* infl_r = nullptr;
      CK(tmp.get(&strong_r, L.nnz));
      CK(tmp.get(&infl_r, n));
      CKH(hipMemsetAsync(infl_r, 0, n * sizeof(int32_t), st));
      hipLaunchKernelGGL(k_strength, g1(n * SG), dim3(256), 0, st, n, L.rowptr, L.col, L.val, prm.theta_r, strong_r,
                         infl_r);
      CKH(hipGetLastError());
    }
    hipLaunchKernelGGL(k_onepoint, grows(n), dim3(256), 0, st, n, blk ? 0 : 1, L.rowptr, L.col, L.val, strong, strong_r, L.cf,
                       cidx, L.pcol, rcnt, clist, L.flist, d_int, d_fst + 2 * l);
    CKH(hipGetLastError());
    if (blk) {
      hipLaunchKernelGGL(k_block_pcol, g1(nbr), dim3(256), 0, st, nbr, (int)L.ob, L.optr, L.ocol, bw, sb, L.cf, cidx,
                         L.pcol);
      CKH(hipGetLastError());
    }
    if (d2) {
      // distance-two neighbourhoods: R row lengths, |N_i| and the R A P bound
      int32_t *mcnt = nullptr, *c2 = nullptr;
      CK(tmp.get(&mcnt, nc));
      CK(tmp.get(&c2, nc));
      hipLaunchKernelGGL(k_lair_count2, dim3((unsigned)nc), dim3(64), 0, st, nc, L.rowptr, L.col, strong_r, L.cf,
                         clist, rcnt, mcnt, c2);
      CKH(hipGetLastError());
      CKH(hipMemsetAsync(d_int, 0, 2 * sizeof(int), st));
      const dim3 gm((unsigned)std::min<int64_t>(cdiv(nc, 256), 256));
      hipLaunchKernelGGL(k_max_i32, gm, dim3(256), 0, st, nc, mcnt, d_int);
      hipLaunchKernelGGL(k_max_i32, gm, dim3(256), 0, st, nc, c2, d_int + 1);
      CKH(hipGetLastError());
    }
    CK(ar.get(&L.Rptr, ncap + 1));
    CK(scan_i32_to_i64(rcnt, L.Rptr, ncap, st, tmp));
    int hmax[4];
    {
      double* pin = pinned_scratch(6);
      if (!pin) { set_error("pinned host allocation failed"); tmp.release(); delete h; return AH_ENOMEM; }
      CKH(hipMemcpyAsync(pin, L.Rptr + ncap, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      CKH(hipMemcpyAsync(pin + 1, d_int, sizeof(hmax), hipMemcpyDeviceToHost, st));
      CKH(hipMemcpyAsync(pin + 3, cidx + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      CKH(hipStreamSynchronize(st));
      std::memcpy(&L.nnzR, pin, sizeof(int64_t));
      std::memcpy(hmax, pin + 1, sizeof(hmax));
      std::memcpy(&nc, pin + 3, sizeof(int64_t));
    }
    if (!d2 && (nc == 0 || (double)nc > prm.stall * (double)n)) {
      // coarsening stalled: this level is the coarsest
      L.pcol = nullptr;
      L.flist = nullptr;
      L.Rptr = nullptr;
      L.nnzR = 0;
      break;
    }
    L.nc = nc;
    L.clist = clist;
    L.fblk = blk;
    if (L.ob) {
      hipLaunchKernelGGL(k_list_vals, grows(n - nc), dim3(256), 0, st, n - nc, L.flist, L.optr, L.ob, d_fst + 64);
      CKH(hipGetLastError());
    }
    CK(ar.get(&L.Rcol, L.nnzR));
    CK(ar.get(&L.Rval, L.nnzR));
    const int maxm = hmax[0];
    // the smallest local-system capacity that holds every neighbourhood
    // (LDS per workgroup, hence occupancy, grows with its square)
    if (maxm > 64) {
      set_error("air_setup: lAIR neighbourhood of %d points exceeds 64", maxm);
      tmp.release(); delete h; return AH_EUNSUPPORTED;
    }
    const int cap = maxm <= 8 ? 8 : maxm <= 16 ? 16 : maxm <= 32 ? 32 : 64;
    if (blk && nc % L.ob) {
      set_error("air_setup: block AIR coarse grid of %lld rows is not made of whole blocks", (long long)nc);
      tmp.release(); delete h; return AH_EUNSUPPORTED;
    }
    if (blk && L.ob <= LB_BMAX) {
      CKH(hipMemsetAsync(d_int + 2, 0, sizeof(int), st));
      CK(lair_blk_dispatch(cap, nc / L.ob, (int)L.ob, L, strong_r, clist, d_ull + 2, d_int + 2, st));
    } else {
      CK(lair_dispatch(cap, d2, nc, L, strong_r, clist, d_ull + 2, st));
    }
    CKH(hipGetLastError());
    // R A P
    const int maxcand = hmax[1];
    int hs = maxcand < 256 ? 256 : maxcand < 512 ? 512 : maxcand < 1024 ? 1024 : maxcand < 2048 ? 2048
                                                     : maxcand < 4096 ? 4096 : -1;
    AhLevel C;
    C.n = nc;
    int32_t* ccnt = nullptr;
    CK(tmp.get(&ccnt, nc + 1));
    // block AIR level 0: the rows of a C block together (a block's
    // candidates: a row's, plus the other b - 1 own rows)
    int hsb = 256;
    while (hsb <= (int64_t)maxcand + (int64_t)(L.ob - 1) * hmax[2] && hsb < 8192) hsb *= 2;
    const bool rblk = blk && rap_blk_fits((int)L.ob, hsb, false) && L.ob <= LB_BMAX;
    if (rblk) CK(rap_blk_dispatch(hsb, (int)L.ob, false, nc / L.ob, L, clist, ccnt, nullptr, nullptr, nullptr, st));
    else CK(rap_dispatch(hs, nc, L, ccnt, nullptr, nullptr, nullptr, false, st));
    CK(ar.get(&C.rowptr, nc + 1));
    CK(scan_i32_to_i64(ccnt, C.rowptr, nc, st, tmp));
    // the numeric pass hashes a row's distinct coarse columns only: size its
    // table from the largest row of A_c
    int rmax = 0;
    {
      hipLaunchKernelGGL(k_max_i32, dim3((unsigned)std::min<int64_t>(cdiv(nc, 256), 256)), dim3(256), 0, st, nc, ccnt,
                         d_int + 3);
      CKH(hipGetLastError());
      double* pin = pinned_scratch(2);
      if (!pin) { set_error("pinned host allocation failed"); tmp.release(); delete h; return AH_ENOMEM; }
      CKH(hipMemcpyAsync(pin, C.rowptr + nc, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      CKH(hipMemcpyAsync(pin + 1, d_int + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      CKH(hipStreamSynchronize(st));
      std::memcpy(&C.nnz, pin, sizeof(int64_t));
      int e2[2];
      std::memcpy(e2, pin + 1, sizeof(e2));
      rmax = e2[1];
      if (blk && e2[0]) {
        set_error("air_setup: rows of a facet block differ in their block AIR neighbourhood");
        tmp.release(); delete h; return AH_EUNSUPPORTED;
      }
    }
    int hsn = 64;
    while (hsn < 2 * rmax && hsn < hs) hsn *= 2;
    // the block pass hashes the union of its rows' columns (at most a row's
    // plus the b - 1 other own columns)
    int hsnb = 64;
    while (hsnb < 2 * (rmax + (int)L.ob) && hsnb < hsb) hsnb *= 2;
    const bool nblk = rblk && rap_blk_fits((int)L.ob, hsnb, true);
    CK(ar.get(&C.col, C.nnz));
    CK(ar.get(&C.val, C.nnz));
    {
      ProfScope ps;
      // algorithmic bytes of the numeric product: R once, the A rows it
      // touches (bounded by the candidate count), P columns, A_c written
      double by = (double)L.nnzR * 12.0 + (double)(nc + 1) * 8.0 + (double)C.nnz * 12.0 + (double)(nc + 1) * 8.0 +
                  (double)L.nnz * 12.0 + (double)n * 4.0;
      prof_begin(ps, l == 0 ? "rap0" : nullptr, st, by);
      if (nblk) CK(rap_blk_dispatch(hsnb, (int)L.ob, true, nc / L.ob, L, clist, ccnt, C.rowptr, C.col, C.val, st));
      else CK(rap_dispatch(hsn, nc, L, ccnt, C.rowptr, C.col, C.val, true, st));
      prof_end(ps);
    }
    if (prm.fp32_cycle) {
      CK(ar.get(&L.Rval32, L.nnzR));
      hipLaunchKernelGGL(k_cast32, g1(L.nnzR), dim3(256), 0, st, L.nnzR, L.Rval, L.Rval32);
      CKH(hipGetLastError());
    }
    if (prm.adjoint && l == 0 && L.ob && prm.relax < 2 && n > tail_max) {
      const int64_t nbr = n / L.ob;
      CK(ar.get(&L.otval, L.nov));
      CKH(hipMemsetAsync(d_int + 2, 0, sizeof(int), st));
      hipLaunchKernelGGL(k_fb_transpose, g1(nbr), dim3(256), 0, st, nbr, L.ob, L.optr, L.ocol, L.oval, L.otval,
                         d_int + 2);
      CKH(hipGetLastError());
      int bad = 0;
      CK(read_bytes(d_int + 2, &bad, sizeof(int), st));
      if (bad) {
        L.otval = nullptr;
      } else {
        at0_csr = false;
        if (prm.fp32_cycle) {
          CK(ar.get(&L.otval32, L.nov));
          hipLaunchKernelGGL(k_cast32, g1(L.nov), dim3(256), 0, st, L.nov, L.otval, L.otval32);
          CKH(hipGetLastError());
        }
      }
    }
    if (prm.adjoint) {
      if (l > 0 || at0_csr)
        CK(transpose(n, n, L.rowptr, L.col, L.val, L.nnz, ar, tmp, st, &L.ATptr, &L.ATcol, &L.ATval));
      CK(transpose(nc, n, L.Rptr, L.Rcol, L.Rval, L.nnzR, ar, tmp, st, &L.RTptr, &L.RTcol, &L.RTval));
      int32_t* pc = nullptr;
      int64_t* pp = nullptr;
      int32_t* pcc = nullptr;
      CK(tmp.get(&pc, n + 1));
      CK(tmp.get(&pp, n + 1));
      hipLaunchKernelGGL(k_p_rowcnt, g1(n), dim3(256), 0, st, n, L.pcol, pc);
      CKH(hipGetLastError());
      CK(scan_i32_to_i64(pc, pp, n, st, tmp));
      int64_t nnzp = 0;
      CK(read_i64(pp + n, &nnzp, st));
      CK(tmp.get(&pcc, nnzp));
      hipLaunchKernelGGL(k_p_fill, g1(n), dim3(256), 0, st, n, L.pcol, pp, pcc);
      CKH(hipGetLastError());
      CK(transpose(n, nc, pp, pcc, nullptr, nnzp, ar, tmp, st, &L.PTptr, &L.PTcol, nullptr));
      L.nnzP = nnzp;
      if (prm.fp32_cycle) {
        if (L.ATval) {
          CK(ar.get(&L.ATval32, L.nnz));
          hipLaunchKernelGGL(k_cast32, g1(L.nnz), dim3(256), 0, st, L.nnz, L.ATval, L.ATval32);
        }
        CK(ar.get(&L.RTval32, L.nnzR));
        hipLaunchKernelGGL(k_cast32, g1(L.nnzR), dim3(256), 0, st, L.nnzR, L.RTval, L.RTval32);
        CKH(hipGetLastError());
      }
    }
    // (the temporary buffers go back to the pool in stream order)
    tmp.release();
    h->lev.push_back(C);
  }
  // coarsest: dense inverse
  AhLevel& LL = h->lev.back();
  const int64_t nL = LL.n;
  if (nL > 8192) {
    set_error("air_setup: coarsest level has %lld points (dense limit 8192)", (long long)nL);
    tmp.release(); delete h; return AH_EUNSUPPORTED;
  }
  if (nL > 0) {
    double* M = nullptr;
    CK(tmp.get(&M, nL * nL));
    CK(ar.get(&h->cinv, nL * nL));
    CKH(hipMemsetAsync(M, 0, nL * nL * sizeof(double), st));
    hipLaunchKernelGGL(k_dense, g1(nL), dim3(256), 0, st, nL, LL.rowptr, LL.col, LL.val, M);
    CKH(hipMemsetAsync(d_int + 2, 0, sizeof(int), st));
    if (nL <= INV_GJ_MAX)
      hipLaunchKernelGGL(k_inv_gj, dim3(1), dim3(256), 0, st, (int)nL, M, h->cinv, d_int + 2);
    else if (nL <= INV_LDS_MAX)
      hipLaunchKernelGGL(k_inv_lds, dim3(1), dim3(1024), 0, st, (int)nL, M, h->cinv, d_int + 2);
    else {
      // many workgroups per column (one workgroup took about 90 ms at
      // n = 480, a stalled coarsening of a pure-advection slab)
      double* fcol = nullptr;
      CK(tmp.get(&fcol, nL));
      hipLaunchKernelGGL(k_eye, g1(nL * nL), dim3(256), 0, st, (int)nL, h->cinv);
      for (int c = 0; c < (int)nL; ++c) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, st, (int)nL, c, M, h->cinv, fcol, d_int + 2);
        hipLaunchKernelGGL(k_gj_update, g1(2 * nL * nL), dim3(256), 0, st, (int)nL, c, M, h->cinv, fcol);
      }
    }
    CKH(hipGetLastError());
  }
  if (prm.adjoint && !h->lev[0].ATptr && !h->lev[0].otval) {
    // level 0 is the coarsest: the adjoint FGMRES still needs S_hat^T
    AhLevel& A0 = h->lev[0];
    CK(transpose(A0.n, A0.n, A0.rowptr, A0.col, A0.val, A0.nnz, ar, tmp, st, &A0.ATptr, &A0.ATcol, &A0.ATval));
  }
  if (prm.relax >= 2) {
    rc = flow_order_build(h, st);
    if (rc < 0) { tmp.release(); delete h; return rc; }
  }
  unsigned long long fb = 0;
  int gerr = 0;
  {
    double* pin = pinned_scratch(70);
    if (!pin) { set_error("pinned host allocation failed"); tmp.release(); delete h; return AH_ENOMEM; }
    CKH(hipMemcpyAsync(pin, d_ull + 2, sizeof(fb), hipMemcpyDeviceToHost, st));
    CKH(hipMemcpyAsync(pin + 1, d_int + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    CKH(hipMemcpyAsync(pin + 2, d_fst, 65 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    CKH(hipMemcpyAsync(pin + 67, d_ull + 3, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    CKH(hipStreamSynchronize(st));
    std::memcpy(&fb, pin, sizeof(fb));
    std::memcpy(&gerr, pin + 1, sizeof(int));
    unsigned long long fst[65];
    std::memcpy(fst, pin + 2, sizeof(fst));
    h->lev[0].novF = (int64_t)fst[64];
    for (size_t l = 0; l + 1 < h->lev.size() && l < 32; ++l) {
      h->lev[l].nF = (int64_t)fst[2 * l];
      h->lev[l].nnzF = (int64_t)fst[2 * l + 1];
    }
    unsigned long long perr = 0;
    std::memcpy(&perr, pin + 67, sizeof(perr));
    if (perr) {
      tmp.release();
      set_error("air_setup: PMIS did not terminate");
      delete h;
      return AH_EINVAL;
    }
  }
  tmp.release();
  if (gerr) {
    set_error("air_setup: singular coarsest matrix");
    delete h;
    return AH_ESINGULAR;
  }
  h->nfallback = (int64_t)fb;
  // tail: the levels from the first one with at most tail_max rows are run
  // by one workgroup inside a single launch per cycle
  {
    if (const char* e = std::getenv("AH_G0")) h->g0 = std::atoi(e);
    if (const char* e = std::getenv("AH_FBB")) h->fbb = std::atoi(e) != 0;
    if (const char* e = std::getenv("AH_LPB")) h->lpb = std::atoi(e);
    if (h->lpb != 2 && h->lpb != 4 && h->lpb != 8) h->lpb = 0;
    if (const char* e = std::getenv("AH_DCGS_MIN")) h->dcgs_min = std::atoll(e);
    if (const char* e = std::getenv("AH_GC")) h->gc = std::atoi(e);
    if (h->gc != 2 && h->gc != 4 && h->gc != 8 && h->gc != 16 && h->gc != 32) h->gc = 0;
    if (const char* e = std::getenv("AH_LIST_MIN")) h->list_min = std::atoll(e);
    if (h->g0 != 2 && h->g0 != 4 && h->g0 != 8 && h->g0 != 16 && h->g0 != 32) h->g0 = 0;
    const int nl = (int)h->lev.size();
    // level 1 under block AIR: R A P with P = P_b (x) I and block lAIR rows
    // is made of ob x ob blocks; its F and C sweeps (list sweeps, not the
    // coarsest level) read it by full blocks (one column index per block)
    bool l1b = true, swo = true, rzb = true;
    if (const char* e = std::getenv("AH_L1B")) l1b = std::atoi(e) != 0;
    if (const char* e = std::getenv("AH_RZB")) rzb = std::atoi(e) != 0;
    if (const char* e = std::getenv("AH_SWO")) swo = std::atoi(e) != 0;
    // level 0 under block AIR with Jacobi sweeps: the sweep-ordered copy
    if (swo && nl > 1 && h->lev[0].fblk && prm.relax < 2 && h->fbb) {
      ProfScope ps;
      prof_begin(ps, "order0", st, 0.0);
      CK(sweep_order_build(h, st));
      prof_end(ps);
    }
    // block AIR: the level-0 restriction by coarse blocks
    if (rzb && nl > 1 && h->lev[0].fblk) {
      ProfScope ps;
      prof_begin(ps, "rz0", st, 0.0);
      CK(rz_build(h, st));
      prof_end(ps);
    }
    // level 0 under scalar AIR with Jacobi sweeps: its rows in sweep order
    if (swo && nl > 1 && !h->lev[0].fblk && h->lev[0].ob && prm.relax < 2) {
      ProfScope ps;
      prof_begin(ps, "order0", st, 0.0);
      CK(row_order_build(h, st));
      prof_end(ps);
    }
    if (l1b && nl > 2 && h->lev[0].fblk && h->lev[1].n >= h->list_min) {
      ProfScope ps;
      prof_begin(ps, "view1", st, 0.0);
      CK(block_view_build(h, 1, h->lev[0].ob, st, swo));
      prof_end(ps);
    }
    // coarse levels swept from their lists without a full-block view: the
    // sweep-ordered CSR copy (not the coarsest level, nor the tail's)
    if (swo)
      for (int l = 1; l + 1 < nl; ++l) {
        if (h->lev[l].n < h->list_min || h->lev[l].bb || h->lev[l].n <= tail_max) continue;
        ProfScope ps;
        prof_begin(ps, "order_csr", st, 0.0);
        CK(csr_order_build(h, l, st));
        prof_end(ps);
      }
    std::vector<TailLevel> tl(nl);
    for (int l = 0; l < nl; ++l) {
      const AhLevel& L = h->lev[l];
      TailLevel& T = tl[l];
      T = TailLevel{};
      T.n = L.n; T.nc = L.nc; T.nnz = L.nnz; T.nnzR = L.nnzR; T.nnzP = L.nnzP;
      T.rp = L.rowptr; T.ci = L.col; T.v = L.val; T.v32 = L.val32; T.d = L.diag; T.d32 = L.diag32;
      T.cf = L.cf; T.pcol = L.pcol;
      T.Rp = L.Rptr; T.Rc = L.Rcol; T.Rv = L.Rval; T.Rv32 = L.Rval32;
      T.ATp = L.ATptr; T.ATc = L.ATcol; T.ATv = L.ATval; T.ATv32 = L.ATval32;
      T.RTp = L.RTptr; T.RTc = L.RTcol; T.RTv = L.RTval; T.RTv32 = L.RTval32;
      T.PTp = L.PTptr; T.PTc = L.PTcol;
      T.b = L.b; T.x = L.x; T.y = L.y; T.b32 = L.b32; T.x32 = L.x32; T.y32 = L.y32;
    }
    // the tail starts at the first level with at most tail_max rows whose
    // levels, down to the coarsest, fit in LDS as an FP64 image
    // (with an ordered relaxation, level 0 is swept outside the tail)
    const int lt = prm.relax >= 2 ? 1 : 0;
    h->tail0 = -1;
    h->tail_lds = false;
    // AH_TAIL_LDS=0 keeps the tail in global memory (both directions)
    bool lds_ok = true;
    if (const char* e = std::getenv("AH_TAIL_LDS")) lds_ok = std::atoi(e) != 0;
    if (lds_ok && nl <= TAIL_MAX_LEVELS) {
      for (int l = lt; l < nl; ++l) {
        if (h->lev[l].n > tail_max) continue;
        TailLds lo[TAIL_MAX_LEVELS];
        int64_t oc = 0;
        const int64_t b64 = tail_lds_layout<8>(tl.data(), l, nl, lo, &oc);
        if (b64 <= TAIL_LDS_MAX) {
          h->tail0 = l;
          h->tail_lds = true;
          h->tail_bytes[0] = b64;
          h->tail_bytes[1] = tail_lds_layout<4>(tl.data(), l, nl, lo, &oc);
          break;
        }
      }
    }
    // the adjoint's transposed tail from an LDS image of the same levels
    if (prm.adjoint && h->tail_lds && nl <= TAIL_MAX_LEVELS) {
      TailLdsT lt_[TAIL_MAX_LEVELS];
      int64_t oc = 0;
      const int64_t b64 = tail_lds_layout_t<8>(tl.data(), h->tail0, nl, lt_, &oc);
      if (b64 <= TAIL_LDS_MAX) {
        h->tail_lds_t = true;
        h->tail_bytes_t[0] = b64;
        h->tail_bytes_t[1] = tail_lds_layout_t<4>(tl.data(), h->tail0, nl, lt_, &oc);
      }
    }
    if (h->tail0 < 0)   // no LDS image fits: small levels run from global memory
      for (int l = lt; l < nl; ++l)
        if (h->lev[l].n <= std::min<int64_t>(tail_max, 500)) { h->tail0 = l; break; }
    rc = ar.get(&h->d_tail, nl);
    if (rc < 0) { delete h; return rc; }
    double* pin = pinned_scratch((nl * sizeof(TailLevel) + 7) / 8);
    if (!pin) { set_error("pinned host allocation failed"); delete h; return AH_ENOMEM; }
    std::memcpy(pin, tl.data(), nl * sizeof(TailLevel));
    if (hipMemcpyAsync(h->d_tail, pin, nl * sizeof(TailLevel), hipMemcpyHostToDevice, st) != hipSuccess) {
      set_error("air_setup: upload of the level table failed");
      delete h;
      return AH_EHIP;
    }
    rc = tail_image_build(h, st);
    if (rc < 0) { delete h; return rc; }
    if (hipStreamSynchronize(st) != hipSuccess) {
      set_error("air_setup: upload of the level table failed");
      delete h;
      return AH_EHIP;
    }
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->levels = (int)h->lev.size();
    double tot = 0;
    for (size_t l = 0; l < h->lev.size() && l < 32; ++l) {
      info->n[l] = h->lev[l].n;
      info->nnz[l] = h->lev[l].nnz;
      tot += (double)h->lev[l].nnz;
    }
    info->n_fallback = h->nfallback;
    info->op_complexity = h->lev[0].nnz ? tot / (double)h->lev[0].nnz : 0.0;
    info->block_view_values = h->lev.size() > 1 ? h->lev[1].nbv : 0;
    info->level0_no_interp_pass = h->lev.size() > 1 && h->lev[0].soce && h->prm.relax == 0 ? 1 : 0;
    info->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  *out = h;
  return AH_OK;
#undef CK
#undef CKH
}

extern "C" void ah_hier_destroy(ah_hier* h) { delete h; }

extern "C" ah_status ah_hier_level_sizes(const ah_hier* h, int l, int64_t* n, int64_t* nnz, int64_t* nnz_r) {
  if (!h || l < 0 || l >= (int)h->lev.size()) { set_error("bad level"); return AH_EINVAL; }
  const AhLevel& L = h->lev[l];
  if (n) *n = L.n;
  if (nnz) *nnz = L.nnz;
  if (nnz_r) *nnz_r = L.nnzR;
  return AH_OK;
}

extern "C" ah_status ah_hier_level_export(const ah_hier* h, int l, int64_t* row_ptr, int32_t* col, double* val,
                                          int8_t* cf, int32_t* pcol, int64_t* r_row_ptr, int32_t* r_col,
                                          double* r_val, void* stream) {
  if (!h || l < 0 || l >= (int)h->lev.size()) { set_error("bad level"); return AH_EINVAL; }
  const AhLevel& L = h->lev[l];
  hipStream_t st = as_stream(stream);
  if (row_ptr) AH_HIP(hipMemcpyAsync(row_ptr, L.rowptr, (L.n + 1) * 8, hipMemcpyDeviceToDevice, st));
  if (col) AH_HIP(hipMemcpyAsync(col, L.col, L.nnz * 4, hipMemcpyDeviceToDevice, st));
  if (val) AH_HIP(hipMemcpyAsync(val, L.val, L.nnz * 8, hipMemcpyDeviceToDevice, st));
  bool coarse = l + 1 < (int)h->lev.size();
  if (coarse) {
    if (cf) AH_HIP(hipMemcpyAsync(cf, L.cf, L.n, hipMemcpyDeviceToDevice, st));
    if (pcol) AH_HIP(hipMemcpyAsync(pcol, L.pcol, L.n * 4, hipMemcpyDeviceToDevice, st));
    if (r_row_ptr) AH_HIP(hipMemcpyAsync(r_row_ptr, L.Rptr, (L.nc + 1) * 8, hipMemcpyDeviceToDevice, st));
    if (r_col) AH_HIP(hipMemcpyAsync(r_col, L.Rcol, L.nnzR * 4, hipMemcpyDeviceToDevice, st));
    if (r_val) AH_HIP(hipMemcpyAsync(r_val, L.Rval, L.nnzR * 8, hipMemcpyDeviceToDevice, st));
  }
  return AH_OK;
}
