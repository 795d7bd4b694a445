// Reconstruction of the element unknowns (Section 2.5), slab coupling
// (Section 2.4), adjoint gradients with respect to the source and nu, and
// Gaussian source fields.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "system.h"

namespace ah {

struct ElemTables;

// Full facet trace of element e's facets: free DOFs from lam (free numbering),
// Dirichlet facets from lamD (or zero when dir_zero).
__device__ inline double trace_at(const int32_t* free_rank, const double* lam, const double* lamD, int f, int m,
                                  int b, bool dir_zero) {
  int fr = free_rank[f];
  if (fr >= 0) return lam[(int64_t)fr * b + m];
  return dir_zero ? 0.0 : lamD[(int64_t)f * b + m];
}

// U_K = A_K^-1 (F_K - B_K Lambda_K), then the values at the element lattice.
__global__ void k_reconstruct(int64_t ne, int D, int nu, int b, const int32_t* __restrict__ elem_facet,
                              const int32_t* __restrict__ free_rank, const double* __restrict__ lam,
                              const double* __restrict__ lamD, const double* __restrict__ Ainv,
                              const double* __restrict__ Bm, const double* __restrict__ Fv,
                              const double* __restrict__ lat_phi, double* __restrict__ U) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int nl = (D + 1) * b;
  double L[40], r[20], u[20];
  for (int lf = 0; lf <= D; ++lf) {
    int f = elem_facet[e * (D + 1) + lf];
    for (int m = 0; m < b; ++m) L[lf * b + m] = trace_at(free_rank, lam, lamD, f, m, b, false);
  }
  for (int i = 0; i < nu; ++i) {
    double s = Fv[e * nu + i];
    for (int c = 0; c < nl; ++c) s -= Bm[(e * nu + i) * nl + c] * L[c];
    r[i] = s;
  }
  for (int i = 0; i < nu; ++i) {
    double s = 0.0;
    for (int k = 0; k < nu; ++k) s += Ainv[(e * nu + i) * nu + k] * r[k];
    u[i] = s;
  }
  for (int k = 0; k < nu; ++k) {
    double s = 0.0;
    for (int i = 0; i < nu; ++i) s += lat_phi[k * nu + i] * u[i];
    U[e * nu + k] = s;
  }
}

// Inflow data of the next slab: g at the facet points = previous trace.
struct FacetLattice {
  int8_t beta[10][3];
};

__global__ void k_inflow(int64_t npair, int D, int p, int b, int nqf, const int32_t* __restrict__ pair,
                         const uint8_t* __restrict__ perm, const double* __restrict__ fac_mu,
                         const int32_t* __restrict__ src_free_rank, const double* __restrict__ lam_prev,
                         const double* __restrict__ lamD_prev, FacetLattice lat, double* __restrict__ g) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npair * nqf) return;
  int64_t k = idx / nqf;
  int q = (int)(idx % nqf);
  int bi = pair[2 * k], f = pair[2 * k + 1];
  double mu[3] = {0, 0, 0};
  for (int s = 0; s < D; ++s) mu[perm[k * D + s]] = fac_mu[q * D + s];
  double v = 0.0;
  for (int m = 0; m < b; ++m) {
    double psi = 1.0;
    for (int s = 0; s < D; ++s)
      for (int j = 0; j < lat.beta[m][s]; ++j) psi *= (p * mu[s] - j) / (j + 1.0);
    v += psi * trace_at(src_free_rank, lam_prev, lamD_prev, f, m, b, false);
  }
  g[(int64_t)bi * nqf + q] = v;
}

template <class T>
__global__ void k_sum_partial(int64_t n, const T* __restrict__ x, double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += (double)x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_final(int nb, const double* __restrict__ partial, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += partial[k];
    *out = s;
  }
}

// f(X) = sum_k c_k exp(-|X - X_k|^2 / (2 w^2))
__global__ void k_gauss(int64_t npts, int D, const double* __restrict__ X, int K, const double* __restrict__ C,
                        double inv2w2, const double* __restrict__ c, double* __restrict__ f) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts) return;
  double x[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) x[a] = X[i * D + a];
  double s = 0.0;
  for (int k = 0; k < K; ++k) {
    double r2 = 0.0;
    for (int a = 0; a < D; ++a) { double d = x[a] - C[k * D + a]; r2 += d * d; }
    s += c[k] * exp(-r2 * inv2w2);
  }
  f[i] = s;
}

// partial[k][blk] = sum over the block's points of y(X) phi_k(X)
__global__ __launch_bounds__(256) void k_gauss_t(int64_t npts, int D, const double* __restrict__ X, int K,
                                                 const double* __restrict__ C, double inv2w2,
                                                 const double* __restrict__ y, double* __restrict__ partial, int nblk) {
  __shared__ double red[256];
  const int k = blockIdx.y;
  double ck[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) ck[a] = C[k * D + a];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npts; i += (int64_t)nblk * 256) {
    double r2 = 0.0;
    for (int a = 0; a < D; ++a) { double d = X[i * D + a] - ck[a]; r2 += d * d; }
    s += y[i] * exp(-r2 * inv2w2);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)k * nblk + blockIdx.x] = red[0];
}

__global__ void k_rows_sum(int K, int nblk, const double* __restrict__ partial, double* __restrict__ out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)k * nblk + b];
  out[k] = s;
}

ah_status grad_dispatch(const ah_system* s, const double* a_vert, const double* lam_fwd, const double* lam_adj,
                        double* dJdf_q, double* dnu_elem, hipStream_t st);

}  // namespace ah

using namespace ah;

extern "C" ah_status hdg_reconstruct(const ah_system* s, const double* lam, double* U, void* stream) {
  if (!s || !lam || !U) { set_error("hdg_reconstruct: null argument"); return AH_EINVAL; }
  if (!s->keep) { set_error("hdg_reconstruct: system assembled without keep_element_data"); return AH_EINVAL; }
  hipStream_t st = as_stream(stream);
  const ah_mesh* m = s->mesh;
  if (m->ne == 0) return AH_OK;
  hipLaunchKernelGGL(k_reconstruct, dim3((unsigned)cdiv(m->ne, 128)), dim3(128), 0, st, m->ne, s->D, s->nu, s->b,
                     m->d_elem_facet, m->d_free_rank, lam, s->d_lamD, s->d_Ainv, s->d_Bm, s->d_Fv, s->tab.d_lat_phi, U);
  AH_LAUNCHED();
  return AH_OK;
}

extern "C" ah_status hdg_inflow_from_trace(const ah_system* prev, const double* lam_prev, ah_mesh* m,
                                           double* g_q_next, void* stream) {
  if (!prev || !lam_prev || !m || !g_q_next) { set_error("hdg_inflow_from_trace: null argument"); return AH_EINVAL; }
  if (prev->D != m->D) { set_error("hdg_inflow_from_trace: dimensions differ"); return AH_EINVAL; }
  hipStream_t st = as_stream(stream);
  AH_TRY(mesh_pair_time_planes(m, prev->mesh, st));
  if (m->npair == 0) return AH_OK;
  FacetLattice lat{};
  std::vector<int> idx;
  lattice(prev->D - 1, prev->p, idx);
  for (int k = 0; k < prev->b; ++k) {
    int s0 = prev->p;
    for (int a = 0; a < prev->D - 1; ++a) { lat.beta[k][a + 1] = (int8_t)idx[k * (prev->D - 1) + a]; s0 -= idx[k * (prev->D - 1) + a]; }
    lat.beta[k][0] = (int8_t)s0;
  }
  hipLaunchKernelGGL(k_inflow, dim3((unsigned)cdiv(m->npair * prev->nqf, 256)), dim3(256), 0, st, m->npair, prev->D,
                     prev->p, prev->b, prev->nqf, m->d_pair, m->d_pair_perm, prev->tab.d_fac_mu,
                     prev->mesh->d_free_rank, lam_prev, prev->d_lamD, lat, g_q_next);
  AH_LAUNCHED();
  return AH_OK;
}

extern "C" ah_status hdg_assemble_grad(const ah_system* s, const double* a_vert, const double* lam_fwd,
                                       const double* lam_adj, double* dJdf_q, double* dJdnu, void* stream) {
  if (!s || !lam_fwd || !lam_adj) { set_error("hdg_assemble_grad: null argument"); return AH_EINVAL; }
  if (!s->keep) { set_error("hdg_assemble_grad: system assembled without keep_element_data"); return AH_EINVAL; }
  hipStream_t st = as_stream(stream);
  const int64_t ne = s->mesh->ne;
  Arena tmp;
  tmp.stream = st;
  double* dnu_e = nullptr;
  AH_TRY(tmp.get(&dnu_e, std::max<int64_t>(ne, 1)));
  AH_TRY(grad_dispatch(s, a_vert, lam_fwd, lam_adj, dJdf_q, dnu_e, st));
  if (dJdnu) {
    const int nb = 256;
    double* part = nullptr;
    double* outd = nullptr;
    AH_TRY(tmp.get(&part, nb));
    AH_TRY(tmp.get(&outd, 1));
    hipLaunchKernelGGL(k_sum_partial<double>, dim3(nb), dim3(256), 0, st, ne, dnu_e, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, st, nb, part, outd);
    AH_LAUNCHED();
    AH_HIP(hipMemcpyAsync(dJdnu, outd, sizeof(double), hipMemcpyDeviceToHost, st));
  }
  AH_HIP(hipStreamSynchronize(st));
  tmp.release();
  return AH_OK;
}

extern "C" ah_status ah_source_gauss(int D, int64_t npts, const double* X, int K, const double* centers, double width,
                                     const double* c, double* f, void* stream) {
  if (!X || !centers || !c || !f || D < 1 || D > 3 || K < 0 || !(width > 0)) {
    set_error("ah_source_gauss: invalid arguments");
    return AH_EINVAL;
  }
  if (npts == 0) return AH_OK;
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(k_gauss, dim3((unsigned)cdiv(npts, 256)), dim3(256), 0, st, npts, D, X, K, centers,
                     1.0 / (2.0 * width * width), c, f);
  AH_LAUNCHED();
  return AH_OK;
}

extern "C" ah_status ah_source_gauss_T(int D, int64_t npts, const double* X, int K, const double* centers,
                                       double width, const double* y, double* dc, void* stream) {
  if (!X || !centers || !y || !dc || D < 1 || D > 3 || K <= 0 || !(width > 0)) {
    set_error("ah_source_gauss_T: invalid arguments");
    return AH_EINVAL;
  }
  hipStream_t st = as_stream(stream);
  int nblk = (int)std::min<int64_t>(512, std::max<int64_t>(1, cdiv(npts, 256 * 8)));
  Arena tmp;
  tmp.stream = st;
  double* part = nullptr;
  AH_TRY(tmp.get(&part, (int64_t)K * nblk));
  hipLaunchKernelGGL(k_gauss_t, dim3(nblk, K), dim3(256), 0, st, npts, D, X, K, centers, 1.0 / (2.0 * width * width),
                     y, part, nblk);
  hipLaunchKernelGGL(k_rows_sum, dim3((unsigned)cdiv(K, 256)), dim3(256), 0, st, K, nblk, part, dc);
  AH_LAUNCHED();
  AH_HIP(hipStreamSynchronize(st));
  tmp.release();
  return AH_OK;
}
