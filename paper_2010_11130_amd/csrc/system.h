// Library objects built on the device: the assembled facet system and the
// AIR hierarchy, plus device utilities shared by the kernels.
#pragma once

#include "common.h"

struct ah_system {
  ah_mesh* mesh = nullptr;
  int D = 0, p = 0, nu = 0, b = 0, nl = 0, nq = 0, nqf = 0;
  double visc = 0.0, alpha = 0.0;
  bool keep = false;
  bool unscaled = false;      // no facet-block scaling (S_hat = S, D_b^-1 = I)
  ah::Arena arena;
  ah::RefTables tab;
  int64_t n = 0;        // free DOFs
  int64_t nfree = 0;    // free facets
  int64_t nnzb = 0;     // blocks of the free-facet pattern
  double* d_bval = nullptr;   // [nnzb][b][b] unscaled S
  double* d_H = nullptr;      // [n] unscaled H after Dirichlet elimination
  double* d_H0 = nullptr;     // [n] the same without the Neumann term
  double* d_Hhat = nullptr;   // [n]
  double* d_Dinv = nullptr;   // [nfree][b][b]
  double* d_lamD = nullptr;   // [nf][b]
  int64_t nnz = 0;            // scaled scalar CSR (level 0)
  int64_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  double* d_val = nullptr;
  // the same operator by off-diagonal facet blocks (scaled systems only; the
  // diagonal blocks of S_hat are the identity): block row R with nb blocks
  // holds [b][nb][b] values from (mesh odb_ptr[R]) b^2 on, so scalar row
  // R b + m is contiguous and its entry (s, c) has column b odb_col[.] + c
  double* d_odv = nullptr;    // [nnzb - nfree][b][b]
  // element data kept for reconstruction and the adjoint
  double* d_Ainv = nullptr;   // [ne][nu][nu]
  double* d_Bm = nullptr;     // [ne][nu][nl]
  double* d_Cm = nullptr;     // [ne][nl][nu]
  double* d_Fv = nullptr;     // [ne][nu]
  ~ah_system() { arena.release(); }
};

namespace ah {

// Build the LDS image of the forward tail in global memory (once per
// hierarchy; the cycle then stages it with one contiguous copy).
ah_status tail_image_build(ah_hier* h, hipStream_t st);
// Flow order of the level-0 facet blocks for the ordered relaxations
// (Lemma 3.1): block levels, blocks and F rows grouped by level.
ah_status flow_order_build(ah_hier* h, hipStream_t st);

// Exclusive prefix sum of n int64 values into out[0..n] (out[n] = total).
ah_status scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t st, Arena& tmp);
// Same for int32 counts producing int64 offsets.
ah_status scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t st, Arena& tmp);
// Read one int64 / a few bytes from the device through the pinned staging
// buffer (synchronizes the stream).
ah_status read_i64(const int64_t* d, int64_t* h, hipStream_t st);
ah_status read_bytes(const void* d, void* h, size_t bytes, hipStream_t st);

constexpr int WAVE = 64;

}  // namespace ah

// Where one row of a coarse level read by full blocks sits in the sweep-ordered
// copy: the row's values from voff, its nb block columns from bcol[o0]; one
// 16-byte load per row.
struct alignas(16) AhRowRec {
  int64_t voff;
  int32_t o0;
  int32_t nb;
};

// One level of the AIR hierarchy (scalar CSR, int64 row offsets).
struct AhLevel {
  int64_t n = 0, nnz = 0;
  int64_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
  double* diag = nullptr;
  float* diag32 = nullptr;
  // coarsening (all but the coarsest level)
  int64_t nc = 0;
  int64_t nF = 0, nnzF = 0;    // F rows and their stored entries
  int8_t* cf = nullptr;        // 1 = C, 0 = F
  int32_t* pcol = nullptr;     // one-point interpolation: coarse column or -1
  int32_t* clist = nullptr;    // fine index of each C point (coarse order)
  int32_t* flist = nullptr;    // fine index of each F point (increasing)
  // level 0 of a scaled system: the operator by off-diagonal facet blocks
  // (identity diagonal blocks), ob = block size, 0 where not available
  int ob = 0;
  bool fblk = false;           // F and C points are whole facet blocks (block AIR): block-row sweeps
  int64_t nov = 0;             // stored values (off-diagonal blocks * ob^2)
  int64_t novF = 0;            // of which in F rows
  const int64_t* optr = nullptr;
  const int32_t* ocol = nullptr;
  const double* oval = nullptr;
  float* oval32 = nullptr;
  // block AIR: a copy of that operator with its block rows in sweep order
  // (the F blocks, then the C blocks, each increasing): item k is block row
  // sperm[k], its blocks at soptr[k] .. soptr[k + 1] of socol / soval
  const int32_t* sperm = nullptr;
  const int64_t* soptr = nullptr;
  // scalar AIR: the values of the listed rows in sweep order instead (the F
  // rows, then the C rows), item k's row at rsoff[k] of soval / soval32
  const int64_t* rsoff = nullptr;
  const int32_t* socol = nullptr;
  const double* soval = nullptr;
  float* soval32 = nullptr;
  // block AIR, for sweeps that read the interpolated correction P e_c from
  // e_c itself (one-point P copies coarse blocks): per block o of the copy,
  // socp[o] the coarse block that P copies into column block socol[o] (-1:
  // none, zero) and soce[o] = the F item of an F column block (its values
  // kept compact), ~(its coarse block) for a C one; soown[k] the coarse
  // block P copies into item k's
  // own block row (-1: none; a C item k >= nbF is coarse block k - nbF, since
  // the C list is in coarse order)
  const int32_t* socp = nullptr;
  const int32_t* soce = nullptr;
  const int32_t* soown = nullptr;
  // the transposed operator in the same layout (adjoint cycle): block (I, J)
  // holds the transpose of block (J, I); null where the CSR A^T is used
  double* otval = nullptr;
  float* otval32 = nullptr;
  // a coarse level made of ob x ob blocks (level 1 under block AIR) read by
  // full blocks: block row R has bptr[R + 1] - bptr[R] blocks with column
  // blocks bcol[bptr[R] ..], row m's values at (m nb + s) bb + c from base
  // bvoff[R] of the CSR values (val / val32) where bvoff[R] >= 0, else from
  // ~bvoff[R] of baux / baux32 (zero-filled blocks); bb = 0 where not built
  int bb = 0;
  int blp = 0;                 // lanes per row of its sweeps (0: by precision)
  int64_t nbv = 0;             // stored values
  int64_t nbvF = 0;            // of which in F rows
  int64_t nbaux = 0;           // of which in the side array
  const int64_t* bptr = nullptr;
  const int32_t* bcol = nullptr;
  const int64_t* bvoff = nullptr;
  const double* baux = nullptr;
  float* baux32 = nullptr;
  // and its rows' values once more in sweep order (the F rows, then the C
  // rows, each in list order): item k's row at bsrec[k].voff of soval /
  // soval32, its block columns at bcol[bsrec[k].o0 ..], bsrec[k].nb of them
  const AhRowRec* bsrec = nullptr;
  // a coarse level swept from its point lists (no full-block view): its
  // rows' entries once more in sweep order (the F rows, then the C rows,
  // each in list order): item k's entries at coptr[k] .. coptr[k + 1] of
  // cocol / coval / coval32
  const int64_t* coptr = nullptr;
  const int32_t* cocol = nullptr;
  const double* coval = nullptr;
  float* coval32 = nullptr;
  // block AIR on level 0: R = [Z I] by coarse blocks, Z's b x b blocks (the
  // neighbourhood F blocks) with row m of coarse block k at
  // (rzptr[k] b + m nb) b, column blocks rzcol; null where not built
  const int64_t* rzptr = nullptr;
  const int32_t* rzcol = nullptr;
  const double* rzval = nullptr;
  float* rzval32 = nullptr;
  int64_t nrz = 0;             // stored values of Z
  int64_t nnzR = 0;
  int64_t* Rptr = nullptr;
  int32_t* Rcol = nullptr;
  double* Rval = nullptr;
  float* Rval32 = nullptr;
  // transposes for the adjoint cycle
  int64_t* ATptr = nullptr;
  int32_t* ATcol = nullptr;
  double* ATval = nullptr;
  float* ATval32 = nullptr;
  int64_t* RTptr = nullptr;    // R^T: rows = fine points
  int32_t* RTcol = nullptr;
  double* RTval = nullptr;
  float* RTval32 = nullptr;
  int64_t* PTptr = nullptr;    // P^T: rows = coarse points, entries = fine points (weight 1)
  int64_t nnzP = 0;
  int32_t* PTcol = nullptr;
  // cycle work vectors; e receives the level's correction from the finer
  // level's recursion, so it never aliases the sweep buffers x and y
  double* b = nullptr;
  double* x = nullptr;
  double* y = nullptr;
  double* e = nullptr;
  float* b32 = nullptr;
  float* x32 = nullptr;
  float* y32 = nullptr;
  float* e32 = nullptr;
};

// Flat copy of a level's device pointers for the single-workgroup kernel
// that runs the coarse end of a V-cycle.
struct TailLevel {
  int64_t n, nc, nnz, nnzR, nnzP;
  const int64_t* rp; const int32_t* ci; const double* v; const float* v32;
  const double* d; const float* d32;
  const int8_t* cf; const int32_t* pcol;
  const int64_t* Rp; const int32_t* Rc; const double* Rv; const float* Rv32;
  const int64_t* ATp; const int32_t* ATc; const double* ATv; const float* ATv32;
  const int64_t* RTp; const int32_t* RTc; const double* RTv; const float* RTv32;
  const int64_t* PTp; const int32_t* PTc;
  double *b, *x, *y;
  float *b32, *x32, *y32;
};

// Byte offsets of one level's arrays in the LDS image of the forward tail
// cycle (row offsets and indices as int32, values and vectors of width W).
struct TailLds {
  int32_t rp, ci, v, d, cf, pc, Rp, Rc, Rv, b, x, y;
};

// Layout of levels l0 .. nlev-1 (the last one is the coarsest: vectors
// only) followed by the coarsest inverse (FP64).  Every array starts on a
// 16-byte boundary.  Returns the total size in bytes.
template <int W>
__host__ __device__ inline int64_t tail_lds_layout(const TailLevel* lv, int l0, int nlev, TailLds* o,
                                                   int64_t* o_cinv) {
  int64_t off = 0;
  auto take = [&off](int64_t bytes) {
    const int64_t r = off;
    off += (bytes + 15) & ~int64_t(15);
    return (int32_t)r;
  };
  for (int l = l0; l < nlev; ++l) {
    const TailLevel& L = lv[l];
    TailLds& q = o[l - l0];
    q = TailLds{};
    q.b = take(L.n * W);
    q.x = take(L.n * W);
    q.y = take(L.n * W);
    if (l < nlev - 1) {
      q.rp = take((L.n + 1) * 4);
      q.ci = take(L.nnz * 4);
      q.v = take(L.nnz * W);
      q.d = take(L.n * W);
      q.cf = take(L.n);
      q.pc = take(L.n * 4);
      q.Rp = take((L.nc + 1) * 4);
      q.Rc = take(L.nnzR * 4);
      q.Rv = take(L.nnzR * W);
    }
  }
  const int64_t nL = lv[nlev - 1].n;
  *o_cinv = take(nL * nL * 8);
  return off;
}

// The same for the transposed tail cycle of the adjoint: A^T, the diagonal,
// C/F flags, P^T (coarse rows) and R^T (fine rows) per level; vectors g
// (input), x and y.
struct TailLdsT {
  int32_t ATp, ATc, ATv, d, cf, PTp, PTc, RTp, RTc, RTv, g, x, y;
};

template <int W>
__host__ __device__ inline int64_t tail_lds_layout_t(const TailLevel* lv, int l0, int nlev, TailLdsT* o,
                                                     int64_t* o_cinv) {
  int64_t off = 0;
  auto take = [&off](int64_t bytes) {
    const int64_t r = off;
    off += (bytes + 15) & ~int64_t(15);
    return (int32_t)r;
  };
  for (int l = l0; l < nlev; ++l) {
    const TailLevel& L = lv[l];
    TailLdsT& q = o[l - l0];
    q = TailLdsT{};
    q.g = take(L.n * W);
    q.x = take(L.n * W);
    q.y = take(L.n * W);
    if (l < nlev - 1) {
      q.ATp = take((L.n + 1) * 4);
      q.ATc = take(L.nnz * 4);
      q.ATv = take(L.nnz * W);
      q.d = take(L.n * W);
      q.cf = take(L.n);
      q.PTp = take((L.nc + 1) * 4);
      q.PTc = take(L.nnzP * 4);
      q.RTp = take((L.n + 1) * 4);
      q.RTc = take(L.nnzR * 4);
      q.RTv = take(L.nnzR * W);
    }
  }
  const int64_t nL = lv[nlev - 1].n;
  *o_cinv = take(nL * nL * 8);
  return off;
}

// Largest LDS image the staged tail kernel may use (160 KiB per workgroup on
// gfx950, less the kernel's static layout table).
constexpr int64_t TAIL_LDS_MAX = 160 * 1024 - 4096;
constexpr int TAIL_MAX_LEVELS = 32;

struct ah_hier {
  const ah_system* sys = nullptr;
  int tail0 = -1;              // first level handled by the single-workgroup tail kernel
  bool tail_lds = false;       // the forward tail runs from an LDS image of its levels
  int64_t tail_bytes[2] = {0, 0};   // size of that image with FP64 / FP32 values
  bool tail_lds_t = false;     // the transposed tail runs from an LDS image too
  int64_t tail_bytes_t[2] = {0, 0};
  const char* tail_img_t[2] = {nullptr, nullptr};
  int g0 = 0;                  // lanes per row of the level-0 kernels (0: from the mean row length)
  int fbb = 1;                 // level-0 kernels by facet block rows where the rows are whole blocks
  int lpb = 0;                 // lanes per block row of those (0: from the mean blocks per row)
  int64_t dcgs_min = (int64_t)1 << 21;   // FGMRES uses delayed CGS2 from this many unknowns on
  int gc = 0;                  // lanes per row of the coarse-level kernels (0: from the mean row length)
  int64_t list_min = (int64_t)1 << 16;   // coarse levels from this many rows on sweep their F and C lists
  TailLevel* d_tail = nullptr; // device copy of every level's pointers
  const char* tail_img[2] = {nullptr, nullptr};   // the tail's LDS image (FP64 / FP32), built at setup
  ah::Arena arena;
  ah_air_params prm{};
  std::vector<AhLevel> lev;
  double* cinv = nullptr;      // dense inverse of the coarsest matrix [nL][nL]
  int64_t nfallback = 0;
  // flow order of the level-0 facet blocks (ordered relaxations): level k
  // holds the blocks ord[ord_lptr[k] .. ord_lptr[k+1]) and the F rows
  // ord_frows[ord_lptrF[k] .. ord_lptrF[k+1])
  int32_t* ord = nullptr;
  int32_t* ord_level = nullptr;  // [blocks] level of each block
  int32_t* ord_frows = nullptr;
  int32_t* ord_cols = nullptr;   // level-0 block columns, ~J where J is on the row's level
  // per position of ord / ord_frows: {block or row, first value slot of the
  // block row, its number of blocks, 0}, so a sweep reads one record per row
  // before its values
  int4* ord_info = nullptr;
  int4* ord_finfo = nullptr;
  std::vector<int64_t> ord_lptr, ord_lptrF;
  int ord_breaks = 0;            // rounds that broke a cycle
  // FGMRES workspace (allocated on first solve)
  int m_alloc = 0;
  double* V = nullptr;         // [(m+1)][n]
  double* Z = nullptr;         // [m][n] (FP64 cycle)
  float* Z32 = nullptr;        // [m][n] (FP32 cycle)
  double* w = nullptr;
  double* r = nullptr;
  double* bhat = nullptr;
  double* bcg = nullptr;       // BiCGSTAB vectors [8][n] (allocated on first use)
  float* bcg32 = nullptr;      // FP32 cycle output [n]
  double* partial = nullptr;   // reduction partials
  double* hdev = nullptr;      // [4 (m+3)] device scalars
  ~ah_hier();
};
