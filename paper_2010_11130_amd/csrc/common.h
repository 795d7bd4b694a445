// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "airhdg.h"

namespace ah {

void set_error(const char* fmt, ...);
const char* g_last_error_cstr();

#define AH_HIP(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::ah::set_error("%s:%d: %s: %s", __FILE__, __LINE__, #call,               \
                      hipGetErrorString(e_));                                   \
      return AH_EHIP;                                                           \
    }                                                                           \
  } while (0)

#define AH_TRY(call)                                                            \
  do {                                                                          \
    ah_status s_ = (call);                                                      \
    if (s_ < 0) return s_;                                                      \
  } while (0)

// Launch check: kernel launch errors surface through hipGetLastError.
#define AH_LAUNCHED()  AH_HIP(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Stream-ordered device memory owned by a library object: requests are
// carved (256-byte aligned) out of chunks of at least CHUNK bytes, so an
// object makes a handful of allocation calls instead of one per buffer.
// Stream-ordered bump allocator: chunks come from the library's caching
// allocator (or the caller's) for the arena's current stream and go back to
// it with the stream each chunk came from.  A chunk is only carved on the
// stream it was allocated on; switching stream starts a new chunk.
struct Arena {
  static constexpr size_t CHUNK = size_t(32) << 20;
  // a chunk with the stream it was allocated on and, for memory from a
  // caller-registered allocator (ah_set_allocator), that allocator's free
  struct Chunk {
    void* p;
    hipStream_t stream;
    size_t bytes;
    ah_free_fn free_fn;
    void* ctx;
    int dev;                         // device of a library-cache chunk
  };
  std::vector<Chunk> ptrs;
  char* cur = nullptr;
  size_t left = 0;
  hipStream_t stream = nullptr;      // stream of the next allocations
  hipStream_t cur_stream = nullptr;  // stream of the chunk being carved
  ah_status alloc(void** p, size_t bytes);
  template <class T>
  ah_status get(T** p, size_t count) {
    return alloc(reinterpret_cast<void**>(p), count * sizeof(T) + 16);
  }
  void release();
};

// Process-wide pinned host staging buffer (grown on demand, never freed)
// for small device-to-host reads.
double* pinned_scratch(size_t doubles);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- sizes
inline int dim_p(int D, int p) {  // dim P_p on a D-simplex
  int r = 1;
  for (int k = 1; k <= D; ++k) r = r * (p + k) / k;
  return D == 0 ? 1 : r;
}

// Host reference data of (D, p): quadrature and basis tables uploaded once.
struct RefTables {
  int D = 0, p = 0, nq = 0, nqf = 0, nu = 0, b = 0;
  // host copies
  std::vector<double> vol_w, vol_lam;         // [nq], [nq][D+1]
  std::vector<double> vol_phi, vol_dphi;      // [nq][nu], [nq][nu][D]  (monomial basis)
  std::vector<double> fac_w, fac_mu;          // [nqf] (sum 1), [nqf][D]
  std::vector<double> fac_psi;                // [nqf][b]
  std::vector<double> fac_proj;               // [b][nqf]  L2 projection onto P_p(F)
  std::vector<int> mono;                      // [nu][D] exponents of the element basis
  std::vector<double> lat_phi;                // [nu lattice nodes][nu] basis at element lattice
  // reference tensors of the volume terms (affine element, velocity linear
  // in each element), by the element rule:
  //   ten_adv[k][r][i][j] = sum_q w_q lam_k phi_j d_r phi_i   (k <= D, r < D)
  //   ten_dif[r][s][i][j] = sum_q w_q d_r phi_j d_s phi_i     (r, s < D)
  std::vector<double> ten_adv, ten_dif;
  // device copies
  double* d_vol_w = nullptr;
  double* d_vol_lam = nullptr;
  double* d_vol_phi = nullptr;
  double* d_vol_dphi = nullptr;
  double* d_fac_w = nullptr;
  double* d_fac_mu = nullptr;
  double* d_fac_psi = nullptr;
  double* d_fac_proj = nullptr;
  double* d_lat_phi = nullptr;
  double* d_ten_adv = nullptr;
  double* d_ten_dif = nullptr;
};

ah_status build_ref_tables(int D, int p, RefTables& t);
ah_status upload_ref_tables(RefTables& t, Arena& arena);
void gauss_jacobi01(int n, double alpha, double* s, double* w);
void simplex_rule(int dim, int n, std::vector<double>& xi, std::vector<double>& w);
void lattice(int dim, int p, std::vector<int>& idx);   // [nn][dim], i_1 fastest

}  // namespace ah

// ------------------------------------------------------------- objects
struct ah_mesh {
  int D = 0;
  int64_t nv = 0, ne = 0, nf = 0, nbf = 0;
  std::vector<double> vert;          // [nv][D]
  std::vector<int32_t> cell;         // [ne][D+1]
  std::vector<int32_t> facet_vert;   // [nf][D] sorted
  std::vector<int32_t> facet_elem;   // [nf][2]
  std::vector<int32_t> elem_facet;   // [ne][D+1]
  std::vector<uint8_t> facet_loc;    // [ne][D+1][D]: local vertex of sorted facet vertex s
  std::vector<int32_t> bfacets;      // boundary facet ids ascending
  std::vector<int32_t> bf_index;     // [nf] -> boundary index or -1
  std::vector<int8_t> kind;          // [nf]
  bool bc_set = false;
  // free-facet numbering and block pattern (after set_bc)
  int64_t nfree = 0;
  std::vector<int32_t> free_rank;    // [nf] -> free facet rank or -1
  std::vector<int64_t> bsr_ptr;      // [nfree+1]
  std::vector<int32_t> bsr_col;      // [nnzb] free facet ranks, sorted per row
  std::vector<int64_t> odb_ptr;      // [nfree+1] the same pattern without the diagonal block
  std::vector<int32_t> odb_col;      // [nnzb - nfree]
  std::vector<int32_t> elem_slot;    // [ne][(D+1)^2] block index or -1
  // time planes and the pairing used for slab coupling: boundary facets of
  // this mesh on t_min matched (by spatial vertex coordinates) with facets on
  // t_max of the mesh pair_src
  double t_min = 0, t_max = 0;
  const ah_mesh* pair_src = nullptr;
  int32_t* d_pair = nullptr;         // dev [npair][2]: (boundary index here, facet id in src)
  uint8_t* d_pair_perm = nullptr;    // dev [npair][D]: src sorted vertex of our sorted vertex s
  int64_t npair = 0;
  // device copies of the topology (uploaded once, hipMalloc'd)
  bool dev_ready = false;
  std::mutex lazy_mu;                // guards the lazily built device data above
  double* d_vert = nullptr;
  int32_t* d_cell = nullptr;
  int32_t* d_elem_facet = nullptr;
  uint8_t* d_facet_loc = nullptr;
  int8_t* d_kind = nullptr;
  int32_t* d_bf_index = nullptr;
  int32_t* d_bfacets = nullptr;
  int32_t* d_facet_vert = nullptr;
  int32_t* d_free_rank = nullptr;
  int32_t* d_elem_slot = nullptr;
  int64_t* d_bsr_ptr = nullptr;
  int32_t* d_bsr_col = nullptr;
  int64_t* d_odb_ptr = nullptr;
  int32_t* d_odb_col = nullptr;
  ~ah_mesh();
};

namespace ah {
ah_status mesh_upload(ah_mesh* m, hipStream_t st);
ah_status mesh_pair_time_planes(ah_mesh* m, const ah_mesh* src, hipStream_t st);
}

struct ah_system;
struct ah_hier;
