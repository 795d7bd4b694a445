// Flow order of the level-0 facet blocks for the ordered Gauss-Seidel
// relaxations (Lemma 3.1, Section 3.3), built on the device.
//
// A coupled pair of off-diagonal blocks (I, J) is oriented along its
// dominant coupling, w_IJ = max |S_hat entries of block (I, J)|, when that
// dominance is clear: J precedes I when w_IJ > ratio w_JI.  Levels come from
// Kahn rounds over the oriented pairs: round k places every block whose
// predecessors are all placed; when blocks remain and none is ready (a
// cycle), the remaining block with the fewest unplaced predecessors (then
// the smallest index) is placed alone.  For pure advection on an acyclic
// element graph the upwind flux couples each pair one way only, the scaled
// matrix is block lower triangular in this order, and a forward sweep in it
// is the exact solve.  The sweep is Gauss-Seidel across levels and Jacobi
// inside a level (a level reads its own blocks' values from before the
// level), one launch per level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "airhdg.h"
#include "system.h"

namespace ah {

namespace {

inline dim3 grid1(int64_t n) { return dim3((unsigned)cdiv(n > 0 ? n : 1, 256)); }

// w[s] = max |value| of off-diagonal block slot s; block row R holds
// [B][nb][B] values from optr[R] B^2 on.
__global__ void k_ord_weights(int64_t nbr, int B, const int64_t* __restrict__ optr, const double* __restrict__ ov,
                              double* __restrict__ w) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= nbr) return;
  const int64_t o0 = optr[R];
  const int nblk = (int)(optr[R + 1] - o0);
  const int64_t len = (int64_t)nblk * B;
  const double* __restrict__ v = ov + o0 * B * B;
  for (int k = 0; k < nblk; ++k) {
    double m = 0.0;
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) m = fmax(m, fabs(v[r * len + (int64_t)k * B + c]));
    w[o0 + k] = m;
  }
}

// dir[s] for slot s of row R with column J: 1 when J precedes R, 2 when R
// precedes J, 0 for a pair left unordered; indeg[R] = predecessors of R.
// A slot without its transposed slot sets *bad.
__global__ void k_ord_orient(int64_t nbr, double ratio, const int64_t* __restrict__ optr,
                             const int32_t* __restrict__ ocol, const double* __restrict__ w,
                             uint8_t* __restrict__ dir, int32_t* __restrict__ indeg, int* __restrict__ bad) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= nbr) return;
  int cnt = 0;
  for (int64_t s = optr[R]; s < optr[R + 1]; ++s) {
    const int32_t J = ocol[s];
    double wr = -1.0;
    for (int64_t t = optr[J]; t < optr[J + 1]; ++t)
      if (ocol[t] == (int32_t)R) { wr = w[t]; break; }
    if (wr < 0.0) { *bad = 1; wr = 0.0; }
    const double ws = w[s];
    const uint8_t d = ws > ratio * wr ? 1 : wr > ratio * ws ? 2 : 0;
    dir[s] = d;
    cnt += d == 1;
  }
  indeg[R] = cnt;
}

// Round state on the device: ds[0] = lo, ds[1] = hi (the current round is
// ord[lo .. hi)), ds[2] = blocks appended for the next round, ds[3] = round.
__global__ void k_ord_init(int64_t nbr, const int32_t* __restrict__ indeg, int32_t* __restrict__ level,
                           int32_t* __restrict__ ord, unsigned long long* __restrict__ ds) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= nbr) return;
  level[R] = -1;
  if (indeg[R] == 0) ord[atomicAdd(ds + 1, 1ull)] = (int32_t)R;
}

// One round: the blocks ord[lo .. hi) take level ds[3]; each successor whose
// last predecessor this is joins the next round at ord[hi ..).  Nothing to
// do when lo == hi (finished, or a cycle for the host to break).
__global__ void k_ord_round(int64_t nbr, const unsigned long long* __restrict__ ds0, const int64_t* __restrict__ optr,
                            const int32_t* __restrict__ ocol, const uint8_t* __restrict__ dir,
                            int32_t* __restrict__ indeg, int32_t* __restrict__ level, int32_t* __restrict__ ord,
                            unsigned long long* __restrict__ next) {
  const int64_t lo = (int64_t)ds0[0], hi = (int64_t)ds0[1];
  if (lo >= hi) return;
  const int k = (int)ds0[3];
  for (int64_t t = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < hi;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t R = ord[t];
    if (R < 0 || (int64_t)R >= nbr) continue;
    level[R] = k;
    for (int64_t s = optr[R]; s < optr[R + 1]; ++s) {
      if (dir[s] != 2) continue;
      const int32_t J = ocol[s];
      if (atomicSub(&indeg[J], 1) == 1 && level[J] < 0) {
        // every block joins a round once, so the appends stay below nbr
        const int64_t q = hi + (int64_t)atomicAdd(next, 1ull);
        if (q < nbr) ord[q] = J;
      }
    }
  }
}

// After a round: record its end in lptr and move to the next round.
__global__ void k_ord_advance(int64_t nbr, unsigned long long* __restrict__ ds, int64_t* __restrict__ lptr) {
  if (threadIdx.x != 0) return;
  const unsigned long long lo = ds[0], hi = ds[1];
  if (lo >= hi) return;
  const unsigned long long k = ds[3];
  lptr[k + 1] = (int64_t)hi;
  const unsigned long long nx = hi + ds[2];
  ds[0] = hi;
  ds[1] = nx < (unsigned long long)nbr ? nx : (unsigned long long)nbr;
  ds[2] = 0;
  ds[3] = k + 1;
}

// Cycle break: the unplaced block with the fewest unplaced predecessors,
// then the smallest index, as one 64-bit key.
__global__ void k_ord_argmin(int64_t nbr, const int32_t* __restrict__ indeg, const int32_t* __restrict__ level,
                             unsigned long long* __restrict__ key) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= nbr || level[R] >= 0) return;
  atomicMin(key, ((unsigned long long)(unsigned)indeg[R] << 32) | (unsigned long long)R);
}

// The chosen block forms the round ord[lo .. lo+1).
__global__ void k_ord_place(int64_t nbr, const unsigned long long* __restrict__ key, int32_t* __restrict__ ord,
                            unsigned long long* __restrict__ ds) {
  if (threadIdx.x != 0) return;
  const unsigned long long lo = ds[0];
  if (lo >= (unsigned long long)nbr) return;
  ord[lo] = *key == ~0ull ? -1 : (int32_t)(*key & 0xffffffffull);
  ds[1] = lo + 1;
}

// F rows of the blocks in order: counts, then the rows themselves.
__global__ void k_ord_fcount(int64_t nbr, int B, const int32_t* __restrict__ ord, const int8_t* __restrict__ cf,
                             int32_t* __restrict__ fc) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nbr) return;
  const int64_t R = ord[p];
  if (R < 0 || R >= nbr) { fc[p] = 0; return; }
  int c = 0;
  for (int m = 0; m < B; ++m) c += cf[R * B + m] == 0;
  fc[p] = c;
}

__global__ void k_ord_frows(int64_t nbr, int B, const int32_t* __restrict__ ord, const int8_t* __restrict__ cf,
                            const int64_t* __restrict__ fpos, int32_t* __restrict__ frows) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nbr) return;
  const int64_t R = ord[p];
  if (R < 0 || R >= nbr) return;
  int64_t j = fpos[p];
  for (int m = 0; m < B; ++m)
    if (cf[R * B + m] == 0) frows[j++] = (int32_t)(R * B + m);
}

// Column blocks of the facet-block layout for the sweeps: ~J where block J
// lies on the row's own level (read from the values before the level), J
// otherwise.
__global__ void k_ord_cols(int64_t nbr, const int64_t* __restrict__ optr, const int32_t* __restrict__ ocol,
                           const int32_t* __restrict__ level, int32_t* __restrict__ out) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= nbr) return;
  const int32_t lr = level[R];
  for (int64_t s = optr[R]; s < optr[R + 1]; ++s) {
    const int32_t J = ocol[s];
    out[s] = level[J] == lr ? ~J : J;
  }
}

// Sweep records: {item, first slot of its block row, blocks in that row, 0}
// where item is a block (ord) or a scalar row (F rows, block size B).
__global__ void k_ord_records(int64_t m, int B, const int32_t* __restrict__ items, const int64_t* __restrict__ optr,
                              int4* __restrict__ rec) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const int32_t it = items[t];
  const int64_t R = B > 1 ? it / B : it;
  const int64_t o0 = optr[R];
  rec[t] = make_int4(it, (int)o0, (int)(optr[R + 1] - o0), 0);
}

__global__ void k_ord_gather(int64_t m, const int64_t* __restrict__ idx, const int64_t* __restrict__ src,
                             int64_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) dst[t] = src[idx[t]];
}

}  // namespace

ah_status flow_order_build(ah_hier* h, hipStream_t st) {
  AhLevel& L = h->lev[0];
  if (!L.ob || !L.oval) {
    set_error("air_setup: the ordered relaxations need the facet-block scaled system");
    return AH_EUNSUPPORTED;
  }
  if (!L.cf) return AH_OK;   // level 0 is the coarsest: no relaxation
  const int B = L.ob;
  const int64_t nbr = L.n / B;
  const int64_t nslot = L.nov / ((int64_t)B * B);
  // the sweep records hold a block row's first slot as a 32-bit offset
  if (nslot > (int64_t)INT32_MAX) {
    set_error("air_setup: ordered relaxation needs fewer than 2^31 off-diagonal facet blocks (%lld)",
              (long long)nslot);
    return AH_EUNSUPPORTED;
  }
  Arena tmp;
  tmp.stream = st;
  ah_status rc = AH_OK;
#define OK_(x) do { rc = (x); if (rc < 0) { tmp.release(); return rc; } } while (0)
#define HIP_(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { set_error("air_setup: %s", hipGetErrorString(e_)); tmp.release(); return AH_EHIP; } } while (0)
  double* w = nullptr;
  uint8_t* dir = nullptr;
  int32_t* indeg = nullptr;
  unsigned long long* ds = nullptr;   // [0..3] round state, [4] asymmetric-pattern flag
  unsigned long long* key = nullptr;
  int64_t* dlp = nullptr;
  OK_(tmp.get(&w, nslot));
  OK_(tmp.get(&dir, nslot));
  OK_(tmp.get(&indeg, nbr));
  OK_(tmp.get(&ds, 5));
  OK_(tmp.get(&key, 1));
  OK_(tmp.get(&dlp, nbr + 2));
  OK_(h->arena.get(&h->ord, nbr));
  OK_(h->arena.get(&h->ord_level, nbr));
  HIP_(hipMemsetAsync(ds, 0, 5 * sizeof(unsigned long long), st));
  HIP_(hipMemsetAsync(dlp, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_ord_weights, grid1(nbr), dim3(256), 0, st, nbr, B, L.optr, L.oval, w);
  hipLaunchKernelGGL(k_ord_orient, grid1(nbr), dim3(256), 0, st, nbr, h->prm.order_ratio, L.optr, L.ocol, w, dir,
                     indeg, reinterpret_cast<int*>(ds + 4));
  hipLaunchKernelGGL(k_ord_init, grid1(nbr), dim3(256), 0, st, nbr, indeg, h->ord_level, h->ord, ds);
  HIP_(hipGetLastError());
  unsigned long long state[5] = {0, 0, 0, 0, 0};
  OK_(read_bytes(ds, state, sizeof(state), st));
  if (state[4]) {
    set_error("air_setup: the facet-block pattern is not structurally symmetric");
    tmp.release();
    return AH_EUNSUPPORTED;
  }
  // rounds are queued in batches on the device state; the host looks at the
  // state between batches and breaks a cycle when a round came out empty
  // (32 rounds per batch; 2 right after a broken cycle, where more breaks
  // tend to follow)
  const dim3 rgrid((unsigned)std::min<int64_t>(cdiv(nbr, 256), 512));
  int breaks = 0;
  int batch = 32;
  int64_t batches = 0;
  for (;;) {
    for (int r = 0; r < batch; ++r) {
      hipLaunchKernelGGL(k_ord_round, rgrid, dim3(256), 0, st, nbr, ds, L.optr, L.ocol, dir, indeg, h->ord_level,
                         h->ord, ds + 2);
      hipLaunchKernelGGL(k_ord_advance, dim3(1), dim3(64), 0, st, nbr, ds, dlp);
    }
    HIP_(hipGetLastError());
    OK_(read_bytes(ds, state, 4 * sizeof(unsigned long long), st));
    if (state[0] == state[1] && state[1] >= (unsigned long long)nbr) break;
    batch = state[0] == state[1] ? 2 : 32;
    // every batch either advances a round or ends in a cycle that is broken
    if (++batches > 2 * nbr + 4) {
      set_error("air_setup: flow order did not terminate");
      tmp.release();
      return AH_EINVAL;
    }
    if (state[0] == state[1]) {
      HIP_(hipMemsetAsync(key, 0xff, sizeof(unsigned long long), st));
      hipLaunchKernelGGL(k_ord_argmin, grid1(nbr), dim3(256), 0, st, nbr, indeg, h->ord_level, key);
      hipLaunchKernelGGL(k_ord_place, dim3(1), dim3(64), 0, st, nbr, key, h->ord, ds);
      HIP_(hipGetLastError());
      ++breaks;
    }
  }
  const int64_t rounds = (int64_t)state[3];
  std::vector<int64_t>& lptr = h->ord_lptr;
  lptr.assign(rounds + 1, 0);
  {
    double* pin = pinned_scratch((size_t)rounds + 1);
    if (!pin) { set_error("pinned host allocation failed"); tmp.release(); return AH_ENOMEM; }
    HIP_(hipMemcpyAsync(pin, dlp, (rounds + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_(hipStreamSynchronize(st));
    std::memcpy(lptr.data(), pin, (rounds + 1) * sizeof(int64_t));
  }
  if (lptr.back() != nbr) {
    set_error("air_setup: flow order lost blocks");
    tmp.release();
    return AH_EINVAL;
  }
  h->ord_breaks = breaks;
  OK_(h->arena.get(&h->ord_cols, nslot));
  hipLaunchKernelGGL(k_ord_cols, grid1(nbr), dim3(256), 0, st, nbr, L.optr, L.ocol, h->ord_level, h->ord_cols);
  HIP_(hipGetLastError());
  // F rows by level
  const int64_t nl = (int64_t)lptr.size();
  int32_t* fc = nullptr;
  int64_t* fpos = nullptr;
  int64_t* dl = nullptr;
  int64_t* dlf = nullptr;
  OK_(tmp.get(&fc, nbr + 1));
  OK_(tmp.get(&fpos, nbr + 1));
  OK_(tmp.get(&dl, nl));
  OK_(tmp.get(&dlf, nl));
  hipLaunchKernelGGL(k_ord_fcount, grid1(nbr), dim3(256), 0, st, nbr, B, h->ord, L.cf, fc);
  HIP_(hipGetLastError());
  OK_(scan_i32_to_i64(fc, fpos, nbr, st, tmp));
  OK_(h->arena.get(&h->ord_frows, L.n - L.nc + 1));
  hipLaunchKernelGGL(k_ord_frows, grid1(nbr), dim3(256), 0, st, nbr, B, h->ord, L.cf, fpos, h->ord_frows);
  double* pin = pinned_scratch((size_t)nl + 1);
  if (!pin) { set_error("pinned host allocation failed"); tmp.release(); return AH_ENOMEM; }
  std::memcpy(pin, lptr.data(), nl * sizeof(int64_t));
  HIP_(hipMemcpyAsync(dl, pin, nl * sizeof(int64_t), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_ord_gather, grid1(nl), dim3(256), 0, st, nl, dl, fpos, dlf);
  HIP_(hipGetLastError());
  HIP_(hipMemcpyAsync(pin, dlf, nl * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_(hipStreamSynchronize(st));
  h->ord_lptrF.assign(nl, 0);
  std::memcpy(h->ord_lptrF.data(), pin, nl * sizeof(int64_t));
  tmp.release();
  if (h->ord_lptrF.back() != L.n - L.nc) {
    set_error("air_setup: flow order lost F rows");
    return AH_EINVAL;
  }
  // sweep records (value slots as int32, checked above)
  const int64_t nF = L.n - L.nc;
  OK_(h->arena.get(&h->ord_info, nbr));
  OK_(h->arena.get(&h->ord_finfo, nF + 1));
  hipLaunchKernelGGL(k_ord_records, grid1(nbr), dim3(256), 0, st, nbr, 1, h->ord, L.optr, h->ord_info);
  if (nF) hipLaunchKernelGGL(k_ord_records, grid1(nF), dim3(256), 0, st, nF, B, h->ord_frows, L.optr, h->ord_finfo);
  HIP_(hipGetLastError());
  return AH_OK;
#undef OK_
#undef HIP_
}

}  // namespace ah

extern "C" ah_status ah_hier_flow_levels(const ah_hier* h, int32_t* level, int64_t* nblocks, int* rounds,
                                         int* breaks) {
  if (!h) { ah::set_error("ah_hier_flow_levels: null hierarchy"); return AH_EINVAL; }
  const int64_t nb = h->ord ? h->lev[0].n / h->lev[0].ob : 0;
  if (nblocks) *nblocks = nb;
  if (rounds) *rounds = h->ord ? (int)h->ord_lptr.size() - 1 : 0;
  if (breaks) *breaks = h->ord_breaks;
  if (level && nb) {
    if (hipMemcpy(level, h->ord_level, nb * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
      ah::set_error("ah_hier_flow_levels: copy failed");
      return AH_EHIP;
    }
  }
  return AH_OK;
}
