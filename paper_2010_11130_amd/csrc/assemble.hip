// hdg_assemble: element blocks of the space-time HDG bilinear form
// (Section 2.3), static condensation (Section 2.5), deterministic scatter
// into the free-facet block pattern, Dirichlet elimination, and the left
// facet-block-diagonal scaling of Section 4 fused into the conversion to the
// scalar CSR matrix used by AIR.  Also reconstruction, slab coupling and
// the adjoint gradient kernel.
//
// One workgroup (one wave) per element.  The element basis is the monomial
// basis xi^alpha on the reference simplex of the cell; facet unknowns use the
// nodal Lagrange basis on the sorted-vertex facet simplex.  Rows = test
// functions, columns = trial functions:
//   A(u,v) = int_K (-u a_hat.grad_hat v + nu grad u.grad v)
//            + sum_F int_F [(a+ + tau) u v - nu (grad u.n) v - nu u (grad v.n)]
//   B(l,v) = sum_F int_F [(a- - tau) l v + nu l (grad v.n)]
//   C(u,m) = sum_F int_F [-(a+ + tau) u m + nu (grad u.n) m]
//   D(l,m) = sum_F int_F [-(a- - tau) l m] + [F Neumann] int_F a+ l m
//   F(v) = int_K f v,  G(m) = [F Neumann] int_F g m
// with a_n = n_t + a.n, a+ = (a_n+|a_n|)/2, a- = (a_n-|a_n|)/2,
// tau = nu alpha / h_K, h_K = |det J|^(1/D); grad = spatial gradient.
#include <cmath>

#include "prof.h"
#include "system.h"

namespace ah {

template <int D, int P>
struct Sz {
  static constexpr int NU = D == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6;
  static constexpr int B = D == 2 ? (P + 1) : (P + 1) * (P + 2) / 2;
  static constexpr int NFc = D + 1;
  static constexpr int NL = NFc * B;
  static constexpr int N1 = P + 2;
  static constexpr int NQ = D == 2 ? N1 * N1 : N1 * N1 * N1;
  static constexpr int NQF = D == 2 ? N1 : N1 * N1;
  static constexpr int NR = NL + 1 + NU;   // right-hand sides of the element solve
};

struct ElemArgs {
  int64_t ne;
  const double* vert;
  const int32_t* cell;
  const int32_t* elem_facet;
  const uint8_t* facet_loc;
  const int8_t* kind;
  const int32_t* bf_index;
  const int32_t* free_rank;
  const int32_t* elem_slot;
  const double* a_vert;
  const double* a_qe;      // velocity at the element quadrature points [ne][nq][D-1], or null
  const double* a_qf;      // velocity at the facet quadrature points [nf][nqf][D-1], or null
  const double* f_q;
  const double* g_q;
  const double* vol_w;
  const double* vol_lam;
  const double* vol_phi;
  const double* vol_dphi;
  const double* fac_w;
  const double* fac_mu;
  const double* fac_psi;
  const double* fac_proj;
  const double* ten_adv;   // [(D+1) D][nu nu] reference advection tensor
  const double* ten_dif;   // [D D][nu nu] reference diffusion tensor
  double nu, alpha;
  double* bval;
  double* H;
  double* lamD;
  double* Ainv;
  double* Bm;
  double* Cm;
  double* Fv;
  int* err;
  // gradient mode
  const double* lam_fwd;   // [n_free] forward solution (Dirichlet traces from lamD)
  const double* lam_adj;   // [n_free] adjoint solution (zero on Dirichlet facets)
  double* dJdf_q;          // [ne][nq]
  double* dnu_elem;        // [ne]
  int8_t mono[20][3];
};

template <int D, int P>
struct ElemSmem {
  using S = Sz<D, P>;
  double X[(D + 1) * D];
  double av[(D + 1) * (D - 1)];
  double Jinv[D * D];
  double absdet, tau;
  double nrm[(D + 1) * D];
  double area[D + 1];
  double eta[(D + 1) * D];
  int fid[D + 1], kindf[D + 1], bidx[D + 1], loc[(D + 1) * D];
  double A[S::NU * S::NU];
  double Bm[S::NU * S::NL];
  double Cm[S::NL * S::NU];
  double Dd[(D + 1) * S::B * S::B];
  double F[S::NU];
  double LD[S::NL];
  double vcoef[(D + 1) * D + D * D];   // beta_kr, then G_rs
  // quadrature scratch of the integration phase
  struct Quad {
    double q_wf[S::NQ];             // W_q f_q at the element points
    union {
      struct {
        double f_phi[S::NQF * S::NU];
        double f_dn[S::NQF * S::NU];
      };
      double beta[S::NQ * D];       // J^-1 (1, a(x_q)) of the volume phase (velocity at points)
    };
    double f_cA[S::NQF], f_cB[S::NQF], f_cD[S::NQF], f_W[S::NQF], f_g[S::NQF];
    double f_psi[S::NQF * S::B];    // facet basis at the facet points (staged)
    double f_proj[S::B * S::NQF];   // facet L2 projection weights (staged)
  };
  Quad qd;
};

// Element geometry: inverse Jacobian, penalty, facet normals/areas.
template <int D, int P>
__device__ void elem_geometry(const ElemArgs& a, ElemSmem<D, P>& sm, int64_t e, double nu_eff, double alpha) {
  const int t = threadIdx.x;
  if (t < (D + 1) * D) {
    int k = t / D, c = t % D;
    sm.X[t] = a.vert[(int64_t)a.cell[e * (D + 1) + k] * D + c];
    sm.loc[t] = a.facet_loc[e * (D + 1) * D + t];
  }
  if (t < (D + 1) * (D - 1)) {
    int k = t / (D - 1), c = t % (D - 1);
    sm.av[t] = a.a_vert ? a.a_vert[(int64_t)a.cell[e * (D + 1) + k] * (D - 1) + c] : 0.0;
  }
  if (t < D + 1) {
    int f = a.elem_facet[e * (D + 1) + t];
    sm.fid[t] = f;
    sm.kindf[t] = a.kind[f];
    sm.bidx[t] = a.bf_index[f];
  }
  __syncthreads();
  if (t == 0) {
    double J[D * D];   // J[r][c] = X[c+1][r] - X[0][r]
    for (int r = 0; r < D; ++r)
      for (int c = 0; c < D; ++c) J[r * D + c] = sm.X[(c + 1) * D + r] - sm.X[r];
    double det;
    double Ji[D * D];
    if (D == 2) {
      det = J[0] * J[3] - J[1] * J[2];
      Ji[0] = J[3] / det; Ji[1] = -J[1] / det; Ji[2] = -J[2] / det; Ji[3] = J[0] / det;
    } else {
      double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
      det = J[0] * c00 + J[1] * c01 + J[2] * c02;
      Ji[0] = c00 / det; Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det; Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
      Ji[3] = c01 / det; Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det; Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
      Ji[6] = c02 / det; Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det; Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    }
    for (int k = 0; k < D * D; ++k) sm.Jinv[k] = Ji[k];
    double ad = fabs(det);
    sm.absdet = ad;
    double h = pow(ad, 1.0 / D);
    sm.tau = nu_eff * alpha / h;
    double fact = D == 2 ? 2.0 : 6.0;
    for (int lf = 0; lf <= D; ++lf) {
      double g[D];
      for (int c = 0; c < D; ++c) {
        double v = 0.0;
        if (lf == 0)
          for (int r = 0; r < D; ++r) v -= Ji[r * D + c];
        else
          v = Ji[(lf - 1) * D + c];
        g[c] = v;
      }
      double gn = 0.0;
      for (int c = 0; c < D; ++c) gn += g[c] * g[c];
      gn = sqrt(gn);
      for (int c = 0; c < D; ++c) sm.nrm[lf * D + c] = -g[c] / gn;
      sm.area[lf] = D * (ad / fact) * gn;
      for (int r = 0; r < D; ++r) {
        double v = 0.0;
        for (int c = 1; c < D; ++c) v += Ji[r * D + c] * sm.nrm[lf * D + c];
        sm.eta[lf * D + r] = v;
      }
    }
    if (!(ad > 0.0) || !isfinite(ad)) atomicOr(a.err, 2);
  }
  __syncthreads();
}

// Monomial xi^alpha and its reference gradient.
template <int D>
__device__ inline double mono_eval(const int8_t* ex, const double* xi, double* dv) {
  double pw[D][4];
  for (int c = 0; c < D; ++c) {
    pw[c][0] = 1.0;
    for (int k = 1; k < 4; ++k) pw[c][k] = pw[c][k - 1] * xi[c];
  }
  double v = 1.0;
  for (int c = 0; c < D; ++c) v *= pw[c][ex[c]];
  for (int c = 0; c < D; ++c) {
    if (ex[c] == 0) { dv[c] = 0.0; continue; }
    double d = (double)ex[c] * pw[c][ex[c] - 1];
    for (int o = 0; o < D; ++o)
      if (o != c) d *= pw[o][ex[o]];
    dv[c] = d;
  }
  return v;
}

// Integrate A, B, C, D (diagonal facet blocks), F, G and the Dirichlet traces.
// advect = false and nu_eff = 1 gives the nu-derivative of the blocks.
template <int D, int P>
__device__ void elem_integrate(const ElemArgs& a, ElemSmem<D, P>& sm, int64_t e, double nu_eff, bool advect,
                               bool data) {
  using S = Sz<D, P>;
  constexpr int NU = S::NU, NL = S::NL, B = S::B, NQ = S::NQ, NQF = S::NQF;
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  for (int k = t; k < NL; k += NT) sm.LD[k] = 0.0;
  // ---- volume terms from the reference tensors (the element map and the
  // velocity are affine on K): with a_k = (1, a at vertex k),
  // beta_kr = (J^-1 a_k)_r and G_rs = sum over the spatial c of
  // Jinv[r][c] Jinv[s][c],
  //   A_ij = |det J| (nu sum_rs G_rs M^rs_ij - sum_kr beta_kr T^kr_ij),
  //   F_i  = sum_q w_q |det J| f(x_q) phi_i(x_q).
  if (t < (D + 1) * D) {
    const int k = t / D, r = t % D;
    double v = 0.0;
    if (advect) {
      v = sm.Jinv[r * D];
      for (int c = 1; c < D; ++c) v += sm.Jinv[r * D + c] * sm.av[k * (D - 1) + c - 1];
    }
    sm.vcoef[t] = v;
  } else if (t < (D + 1) * D + D * D) {
    const int u = t - (D + 1) * D, r = u / D, s2 = u % D;
    double g = 0.0;
    for (int c = 1; c < D; ++c) g += sm.Jinv[r * D + c] * sm.Jinv[s2 * D + c];
    sm.vcoef[t] = g;
  }
  const bool has_f = data && a.f_q;
  if (has_f)
    for (int q = t; q < NQ; q += NT) sm.qd.q_wf[q] = a.vol_w[q] * sm.absdet * a.f_q[e * NQ + q];
  // velocity given at the quadrature points: beta_q = J^-1 (1, a(x_q)), and
  // the advective part of A_ij is sum_q w_q phi_j(x_q) beta_q . grad phi_i(x_q)
  const bool aq = advect && a.a_qe;
  if (aq)
    for (int k = t; k < NQ * D; k += NT) {
      const int q = k / D, r = k % D;
      double v = sm.Jinv[r * D];
      for (int c = 1; c < D; ++c) v += sm.Jinv[r * D + c] * a.a_qe[((int64_t)e * NQ + q) * (D - 1) + c - 1];
      sm.qd.beta[k] = v;
    }
  __syncthreads();
  for (int idx = t; idx < NU * NU; idx += NT) {
    double adv = 0.0, dif = 0.0;
    if (aq) {
      const int i = idx / NU, j = idx % NU;
      for (int q = 0; q < NQ; ++q) {
        double g = 0.0;
        _Pragma("unroll") for (int r = 0; r < D; ++r) g += sm.qd.beta[q * D + r] * a.vol_dphi[(q * NU + i) * D + r];
        adv += a.vol_w[q] * a.vol_phi[q * NU + j] * g;
      }
    } else {
      _Pragma("unroll") for (int kr = 0; kr < (D + 1) * D; ++kr)
        adv += sm.vcoef[kr] * a.ten_adv[(size_t)kr * NU * NU + idx];
    }
    _Pragma("unroll") for (int rs = 0; rs < D * D; ++rs)
      dif += sm.vcoef[(D + 1) * D + rs] * a.ten_dif[(size_t)rs * NU * NU + idx];
    sm.A[idx] = sm.absdet * (nu_eff * dif - adv);
  }
  __syncthreads();
  for (int i = t; i < NU; i += NT) {
    double acc = 0.0;
    if (has_f)
      for (int q = 0; q < NQ; ++q) acc += sm.qd.q_wf[q] * a.vol_phi[q * NU + i];
    sm.F[i] = acc;
  }
  __syncthreads();
  // ---- facet terms
  for (int k = t; k < NQF * B; k += NT) {
    sm.qd.f_psi[k] = a.fac_psi[k];
    sm.qd.f_proj[k] = a.fac_proj[k];
  }
  for (int lf = 0; lf <= D; ++lf) {
    const bool isN = sm.kindf[lf] == 2;
    const bool isD = sm.kindf[lf] == 1;
    {
      constexpr int FPART = (NQF * 4 <= 64) ? 4 : (NQF * 2 <= 64 ? 2 : 1);
      constexpr int FIPP = (NU + FPART - 1) / FPART;
      for (int idx = t; idx < NQF * FPART; idx += NT) {
        const int q = idx % NQF, part = idx / NQF;
        double lam[D + 1];
        for (int k = 0; k <= D; ++k) lam[k] = 0.0;
        for (int s2 = 0; s2 < D; ++s2) lam[sm.loc[lf * D + s2]] = a.fac_mu[q * D + s2];
        double xi[D];
        for (int c = 0; c < D; ++c) xi[c] = lam[c + 1];
        for (int ii = 0; ii < FIPP; ++ii) {
          const int i = part * FIPP + ii;
          if (i >= NU) break;
          double dv[D];
          double v = mono_eval<D>(a.mono[i], xi, dv);
          double dn = 0.0;
          for (int c = 0; c < D; ++c) dn += dv[c] * sm.eta[lf * D + c];
          sm.qd.f_phi[q * NU + i] = v;
          sm.qd.f_dn[q * NU + i] = dn;
        }
      }
    }
    for (int q = t; q < NQF; q += NT) {
      double lam[D + 1];
      for (int k = 0; k <= D; ++k) lam[k] = 0.0;
      for (int s = 0; s < D; ++s) lam[sm.loc[lf * D + s]] = a.fac_mu[q * D + s];
      double an = 0.0;
      if (advect) {
        an = sm.nrm[lf * D];
        for (int c = 1; c < D; ++c) {
          double v = 0.0;
          if (a.a_qf)
            v = a.a_qf[((int64_t)sm.fid[lf] * NQF + q) * (D - 1) + c - 1];
          else
            for (int k = 0; k <= D; ++k) v += lam[k] * sm.av[k * (D - 1) + c - 1];
          an += v * sm.nrm[lf * D + c];
        }
      }
      double ap = 0.5 * (an + fabs(an)), am = 0.5 * (an - fabs(an));
      double W = a.fac_w[q] * sm.area[lf];
      sm.qd.f_W[q] = W;
      sm.qd.f_cA[q] = W * (ap + sm.tau);
      sm.qd.f_cB[q] = W * (am - sm.tau);
      sm.qd.f_cD[q] = -W * (am - sm.tau) + ((isN && advect) ? W * ap : 0.0);
      sm.qd.f_g[q] = (data && a.g_q && sm.bidx[lf] >= 0) ? a.g_q[(int64_t)sm.bidx[lf] * NQF + q] : 0.0;
    }
    __syncthreads();
    for (int idx = t; idx < NU * NU; idx += NT) {
      int i = idx / NU, j = idx % NU;
      double acc = 0.0;
      _Pragma("unroll 4") for (int q = 0; q < NQF; ++q) {
        double pi = sm.qd.f_phi[q * NU + i], pj = sm.qd.f_phi[q * NU + j];
        acc += sm.qd.f_cA[q] * pj * pi - nu_eff * sm.qd.f_W[q] * (sm.qd.f_dn[q * NU + j] * pi + pj * sm.qd.f_dn[q * NU + i]);
      }
      sm.A[idx] += acc;
    }
    for (int idx = t; idx < NU * B; idx += NT) {
      int i = idx / B, m = idx % B;
      double acc = 0.0;
      _Pragma("unroll 4") for (int q = 0; q < NQF; ++q) {
        double psi = sm.qd.f_psi[q * B + m];
        acc += sm.qd.f_cB[q] * psi * sm.qd.f_phi[q * NU + i] + nu_eff * sm.qd.f_W[q] * psi * sm.qd.f_dn[q * NU + i];
      }
      sm.Bm[i * NL + lf * B + m] = acc;
    }
    for (int idx = t; idx < B * NU; idx += NT) {
      int m = idx / NU, j = idx % NU;
      double acc = 0.0;
      _Pragma("unroll 4") for (int q = 0; q < NQF; ++q) {
        double psi = sm.qd.f_psi[q * B + m];
        acc += -sm.qd.f_cA[q] * sm.qd.f_phi[q * NU + j] * psi + nu_eff * sm.qd.f_W[q] * sm.qd.f_dn[q * NU + j] * psi;
      }
      sm.Cm[(lf * B + m) * NU + j] = acc;
    }
    for (int idx = t; idx < B * B; idx += NT) {
      int m = idx / B, n = idx % B;
      double acc = 0.0;
      _Pragma("unroll 4") for (int q = 0; q < NQF; ++q) acc += sm.qd.f_cD[q] * sm.qd.f_psi[q * B + m] * sm.qd.f_psi[q * B + n];
      sm.Dd[lf * B * B + idx] = acc;
    }
    if (data) {
      for (int m = t; m < B; m += NT) {
        if (isD) {
          double acc = 0.0;
          _Pragma("unroll 4") for (int q = 0; q < NQF; ++q) acc += sm.qd.f_proj[m * NQF + q] * sm.qd.f_g[q];
          sm.LD[lf * B + m] = acc;
        }
      }
    }
    __syncthreads();
  }
}

// Value of a double in lane src (uniform) for the whole wave.
__device__ inline double wave_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ inline int wave_bcast(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

template <int D, int P>
__global__ __launch_bounds__(64) void k_element(ElemArgs a) {
  using S = Sz<D, P>;
  constexpr int NU = S::NU, NL = S::NL, B = S::B, NR = S::NR;
  // columns of [A | B F I], lane l holds columns l + 64 u
  constexpr int NC = NU + NR;
  constexpr int CPL = (NC + 63) / 64;
  __shared__ ElemSmem<D, P> sm;
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  elem_geometry<D, P>(a, sm, e, a.nu, a.alpha);
  elem_integrate<D, P>(a, sm, e, a.nu, true, true);
  // keep the unfactored blocks
  if (a.Bm) {
    for (int k = t; k < NU * NL; k += NT) a.Bm[e * NU * NL + k] = sm.Bm[k];
    for (int k = t; k < NL * NU; k += NT) a.Cm[e * NL * NU + k] = sm.Cm[k];
    for (int k = t; k < NU; k += NT) a.Fv[e * NU + k] = sm.F[k];
  }
  // Gauss-Jordan with partial pivoting on [A | B F I] in registers: the
  // pivot row and the pivot column are broadcast from the lane holding
  // column k; no barriers.  Afterwards the columns right of A hold
  // X = A^-1 [B | F | I].
  double col[CPL][NU];
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int c = t + 64 * u;
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      double v = 0.0;
      if (c < NU) v = sm.A[r * NU + c];
      else if (c < NU + NL) v = sm.Bm[r * NL + (c - NU)];
      else if (c == NU + NL) v = sm.F[r];
      else if (c < NC) v = (r == c - NU - NL - 1) ? 1.0 : 0.0;
      col[u][r] = v;
    }
  }
  bool singular = false;
  for (int k = 0; k < NU; ++k) {
    // pivot search in column k (lane k, slot 0): first largest |a_rk|, r >= k
    double best = -1.0;
    int p = k;
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      const double v = fabs(col[0][r]);
      if (r >= k && v > best) { best = v; p = r; }
    }
    p = wave_bcast(p, k);
    best = wave_bcast(best, k);
    if (!(best > 0.0) || !isfinite(best)) singular = true;
    // swap rows k and p (selects keep the register indices static)
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      double vk = 0.0, vp = 0.0;
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        vk = (r == k) ? col[u][r] : vk;
        vp = (r == p) ? col[u][r] : vp;
      }
#pragma unroll
      for (int r = 0; r < NU; ++r) col[u][r] = (r == k) ? vp : ((r == p) ? vk : col[u][r]);
    }
    // the pivot column, now in lane k
    double f[NU];
#pragma unroll
    for (int r = 0; r < NU; ++r) f[r] = wave_bcast(col[0][r], k);
    double piv = 0.0;
#pragma unroll
    for (int r = 0; r < NU; ++r) piv = (r == k) ? f[r] : piv;
    const double inv = 1.0 / piv;
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      double xk = 0.0;
#pragma unroll
      for (int r = 0; r < NU; ++r) xk = (r == k) ? col[u][r] : xk;
      xk *= inv;
#pragma unroll
      for (int r = 0; r < NU; ++r) col[u][r] = (r == k) ? xk : col[u][r] - f[r] * xk;
    }
  }
  if (singular && t == 0) atomicOr(a.err, 1);
  // Dirichlet part: w = A^-1 B[:, Dir] lambda_D (broadcast from the lanes of
  // the Dirichlet columns), then y = A^-1 F - w
  double w[NU];
#pragma unroll
  for (int r = 0; r < NU; ++r) w[r] = 0.0;
  for (int lf = 0; lf <= D; ++lf) {
    if (sm.kindf[lf] != 1) continue;
    for (int m = 0; m < B; ++m) {
      const int c = NU + lf * B + m;
      const int src = c & 63, us = c >> 6;
      const double ld = sm.LD[lf * B + m];
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        double v = col[0][r];
#pragma unroll
        for (int u = 1; u < CPL; ++u) v = (us == u) ? col[u][r] : v;
        w[r] += wave_bcast(v, src) * ld;
      }
    }
  }
  double y[NU];
  {
    const int c = NU + NL;
    const int src = c & 63, us = c >> 6;
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      double v = col[0][r];
#pragma unroll
      for (int u = 1; u < CPL; ++u) v = (us == u) ? col[u][r] : v;
      y[r] = wave_bcast(v, src) - w[r];
    }
  }
  // S_K = D_K - C_K A^-1 B_K column by column (lane of column NU + cc),
  // scattered at once: <= 2 contributions per entry, so the atomic sums are
  // order-independent
  const int32_t* slot = a.elem_slot + e * (D + 1) * (D + 1);
#pragma unroll
  for (int u = 0; u < CPL; ++u) {
    const int cc = t + 64 * u - NU;
    if (cc < 0 || cc >= NL) continue;
    const int cb = cc / B, cm = cc % B;
    for (int r = 0; r < NL; ++r) {
      const int rb = r / B, rm = r % B;
      double v = (rb == cb) ? sm.Dd[rb * B * B + rm * B + cm] : 0.0;
#pragma unroll
      for (int k = 0; k < NU; ++k) v -= sm.Cm[r * NU + k] * col[u][k];
      const int sl = slot[rb * (D + 1) + cb];
      if (sl >= 0) unsafeAtomicAdd(&a.bval[(int64_t)sl * B * B + rm * B + cm], v);
    }
  }
  // H_K = -C_K (A^-1 F - A^-1 B[:,Dir] lambda_D) - D_K[:,Dir] lambda_D
  for (int r = t; r < NL; r += NT) {
    const int lf = r / B, rm = r % B;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < NU; ++k) v -= sm.Cm[r * NU + k] * y[k];
    if (sm.kindf[lf] == 1)
      for (int n = 0; n < B; ++n) v -= sm.Dd[lf * B * B + rm * B + n] * sm.LD[lf * B + n];
    const int f = sm.fid[lf];
    const int fr = a.free_rank[f];
    if (fr >= 0) unsafeAtomicAdd(&a.H[(int64_t)fr * B + rm], v);
    if (sm.kindf[lf] == 1) a.lamD[(int64_t)f * B + rm] = sm.LD[r];
  }
  // kept element inverse: the identity columns now hold A^-1
  if (a.Ainv) {
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int ci = t + 64 * u - NU - NL - 1;
      if (ci < 0 || ci >= NU) continue;
#pragma unroll
      for (int r = 0; r < NU; ++r) a.Ainv[e * NU * NU + r * NU + ci] = col[u][r];
    }
  }
}

// Inverse of each free facet's diagonal block (Gauss-Jordan, partial
// pivoting).  All register arrays are indexed with compile-time indices
// (unrolled loops, predicated row swaps) so they stay in registers.
template <int B>
__global__ __launch_bounds__(64) void k_diag_inv(int64_t nfree, const int64_t* __restrict__ bptr, const int32_t* __restrict__ bcol,
                           const double* __restrict__ bval, double* __restrict__ dinv, int* err) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nfree) return;
  int64_t s = -1;
  for (int64_t k = bptr[r]; k < bptr[r + 1]; ++k)
    if (bcol[k] == r) { s = k; break; }
  double M[B][B], I[B][B];
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) {
      M[i][j] = s >= 0 ? bval[s * B * B + i * B + j] : 0.0;
      I[i][j] = i == j ? 1.0 : 0.0;
    }
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) scale = fmax(scale, fabs(M[i][j]));
  bool bad = !(scale > 0.0) || !isfinite(scale);
#pragma unroll
  for (int c = 0; c < B; ++c) {
    int p = c;
    double best = fabs(M[c][c]);
#pragma unroll
    for (int q = c + 1; q < B; ++q)
      if (fabs(M[q][c]) > best) { best = fabs(M[q][c]); p = q; }
    if (!(best > 1e-14 * scale)) bad = true;
#pragma unroll
    for (int q = c + 1; q < B; ++q) {
      if (q == p) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
          double x = M[c][j]; M[c][j] = M[q][j]; M[q][j] = x;
          x = I[c][j]; I[c][j] = I[q][j]; I[q][j] = x;
        }
      }
    }
    double d = M[c][c];
    if (d == 0.0) d = 1.0;
    const double inv = 1.0 / d;
#pragma unroll
    for (int j = 0; j < B; ++j) { M[c][j] *= inv; I[c][j] *= inv; }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (q == c) continue;
      const double f = M[q][c];
#pragma unroll
      for (int j = 0; j < B; ++j) { M[q][j] -= f * M[c][j]; I[q][j] -= f * I[c][j]; }
    }
  }
  if (bad) atomicOr(err, 4);
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) dinv[r * B * B + i * B + j] = I[i][j];
}

// Scalar CSR of the level-0 operator on the structural pattern of the free
// facets (entries that happen to be zero are kept).  Scaled system: row
// R*B+m of D_b^-1 S, whose diagonal block is the identity, so the row holds
// its diagonal entry 1 and the B entries of every off-diagonal block, in
// column order; unscaled: the B entries of every block of S, the diagonal
// block included.  Row offsets follow from the block pattern (scaled:
// B R + B^2 odb_ptr[R] for the block row, 1 + B (nb - 1) per row).
template <int B>
__global__ void k_scaled_rowptr(int64_t nfree, const int64_t* __restrict__ bptr,
                                const int64_t* __restrict__ optr, int unscaled, int64_t* __restrict__ rowptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = nfree * B;
  if (i > n) return;
  const int64_t R = i / B;
  const int m = (int)(i - R * B);
  if (unscaled) {
    const int64_t nb = R < nfree ? bptr[R + 1] - bptr[R] : 0;
    rowptr[i] = (int64_t)B * B * bptr[R] + (int64_t)m * B * nb;
  } else {
    const int64_t nob = R < nfree ? optr[R + 1] - optr[R] : 0;
    rowptr[i] = (int64_t)B * R + (int64_t)B * B * optr[R] + (int64_t)m * (1 + B * nob);
  }
}

// One wave per block row R: lane c takes column c of the block row (block
// c/B, node c%B), reads that column of S's block once and writes its B
// scaled entries into the B scalar rows, and into the off-diagonal
// facet-block copy (oval, scaled systems).
template <int B>
__global__ __launch_bounds__(256) void k_csr_scaled(int64_t nfree, const int64_t* __restrict__ bptr,
                                                    const int32_t* __restrict__ bcol, const double* __restrict__ bval,
                                                    const double* __restrict__ dinv, int32_t* __restrict__ col,
                                                    double* __restrict__ val, int unscaled,
                                                    const int64_t* __restrict__ optr, double* __restrict__ oval) {
  const int64_t R = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (R >= nfree) return;
  const int64_t s0 = bptr[R];
  const int nb = (int)(bptr[R + 1] - s0);
  const int64_t o0 = unscaled ? 0 : optr[R];
  const int nob = unscaled ? 0 : (int)(optr[R + 1] - o0);
  // first entry of the block row and the length of each of its rows
  const int64_t base = unscaled ? (int64_t)B * B * s0 : (int64_t)B * R + (int64_t)B * B * o0;
  const int rlen = unscaled ? B * nb : 1 + B * nob;
  for (int c = lane; c < nb * B; c += 64) {
    const int j = c / B, n = c % B;
    const int64_t s = s0 + j;
    const int32_t C = bcol[s];
    double bc[B];
#pragma unroll
    for (int k = 0; k < B; ++k) bc[k] = bval[s * B * B + k * B + n];
#pragma unroll
    for (int m = 0; m < B; ++m) {
      const int64_t rs = base + (int64_t)m * rlen;
      if (unscaled) {
        col[rs + c] = (int32_t)(C * B + n);
        val[rs + c] = bc[m];
      } else if (C == R) {
        if (n == m) {
          col[rs + j * B] = (int32_t)(R * B + m);
          val[rs + j * B] = 1.0;
        }
      } else {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < B; ++k) v += dinv[R * B * B + m * B + k] * bc[k];
        // one diagonal entry precedes the blocks after the diagonal block
        const int pos = C < R ? c : c - B + 1;
        col[rs + pos] = (int32_t)(C * B + n);
        val[rs + pos] = v;
        const int jo = C < R ? j : j - 1;
        oval[o0 * B * B + (int64_t)m * nob * B + jo * B + n] = v;
      }
    }
  }
}

template <int B>
__global__ void k_ident_blocks(int64_t nfree, double* __restrict__ dinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfree * B * B) return;
  const int k = (int)(i % (B * B));
  dinv[i] = (k / B == k % B) ? 1.0 : 0.0;
}

template <int B>
__global__ void k_hhat(int64_t nfree, const double* __restrict__ dinv, const double* __restrict__ H,
                       double* __restrict__ hhat) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfree * B) return;
  int64_t R = i / B;
  int m = (int)(i % B);
  double v = 0.0;
  for (int k = 0; k < B; ++k) v += dinv[R * B * B + m * B + k] * H[R * B + k];
  hhat[i] = v;
}

// Neumann term of the right-hand side (Section 2.3, the data term on the
// initial plane and on Neumann facets): H = H0 + G with
// G_f[m] = |F| sum_q w_q g_q psi_m(x_q) on every free boundary facet of
// Neumann kind.  |F| from the Gram determinant of the facet's edges; the
// facet rule weights sum to one.  One thread per (boundary facet, node);
// each free facet occurs once, so the updates do not collide.
template <int B>
__global__ void k_neumann(int64_t nbf, int D, int nqf, const int32_t* __restrict__ bfacets,
                          const int8_t* __restrict__ kind, const int32_t* __restrict__ free_rank,
                          const int32_t* __restrict__ facet_vert, const double* __restrict__ vert,
                          const double* __restrict__ fac_w, const double* __restrict__ fac_psi,
                          const double* __restrict__ g_q, double* __restrict__ H) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbf * B) return;
  const int64_t bf = idx / B;
  const int m = (int)(idx % B);
  const int32_t f = bfacets[bf];
  if (kind[f] != 2) return;
  const int32_t fr = free_rank[f];
  if (fr < 0) return;
  double X[3][3];
  for (int s = 0; s < D; ++s)
    for (int c = 0; c < D; ++c) X[s][c] = vert[(int64_t)facet_vert[(int64_t)f * D + s] * D + c];
  double area;
  if (D == 2) {
    double e0 = X[1][0] - X[0][0], e1 = X[1][1] - X[0][1];
    area = sqrt(e0 * e0 + e1 * e1);
  } else {
    double u[3], v[3];
    for (int c = 0; c < 3; ++c) { u[c] = X[1][c] - X[0][c]; v[c] = X[2][c] - X[0][c]; }
    double g00 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double g11 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double g01 = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    area = 0.5 * sqrt(fmax(g00 * g11 - g01 * g01, 0.0));
  }
  double acc = 0.0;
  for (int q = 0; q < nqf; ++q) acc += fac_w[q] * g_q[bf * nqf + q] * fac_psi[q * B + m];
  H[(int64_t)fr * B + m] += area * acc;
}

// Physical quadrature points (element rule and boundary-facet rule).
__global__ void k_quad_points_elem(int64_t ne, int D, int nq, const double* __restrict__ vert,
                                   const int32_t* __restrict__ cell, const double* __restrict__ lam,
                                   double* __restrict__ xq) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne * nq) return;
  int64_t e = idx / nq;
  int q = (int)(idx % nq);
  for (int c = 0; c < D; ++c) {
    double v = 0.0;
    for (int k = 0; k <= D; ++k) v += lam[q * (D + 1) + k] * vert[(int64_t)cell[e * (D + 1) + k] * D + c];
    xq[idx * D + c] = v;
  }
}

__global__ void k_quad_points_bfacet(int64_t nbf, int D, int nqf, const double* __restrict__ vert,
                                     const int32_t* __restrict__ bfacets, const int32_t* __restrict__ fvert,
                                     const double* __restrict__ mu, double* __restrict__ xq) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nbf * nqf) return;
  int64_t k = idx / nqf;
  int q = (int)(idx % nqf);
  int64_t f = bfacets[k];
  for (int c = 0; c < D; ++c) {
    double v = 0.0;
    for (int s = 0; s < D; ++s) v += mu[q * D + s] * vert[(int64_t)fvert[f * D + s] * D + c];
    xq[idx * D + c] = v;
  }
}

// Adjoint gradient per element: with U = A^-1 (F - B Lambda) and
// w = -A^-T C^T lam, the derivative of J through F_K at the volume
// quadrature points, W_q w . phi(x_q), and the nu-derivative
// -w.(A1 U + B1 Lambda) - lam.(C1 U + D1 Lambda) with X1 = dX/dnu.
template <int D, int P>
__global__ __launch_bounds__(64) void k_grad(ElemArgs a) {
  using S = Sz<D, P>;
  constexpr int NU = S::NU, NL = S::NL, B = S::B, NQ = S::NQ;
  __shared__ ElemSmem<D, P> sm;
  __shared__ double sL[NL], sLa[NL], sR[NU], sU[NU], sT[NU], sW[NU], sred[64];
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  elem_geometry<D, P>(a, sm, e, 1.0, a.alpha);
  elem_integrate<D, P>(a, sm, e, 1.0, false, false);
  const double* Ai = a.Ainv + e * NU * NU;
  const double* Bo = a.Bm + e * NU * NL;
  const double* Co = a.Cm + e * NL * NU;
  const double* Fo = a.Fv + e * NU;
  for (int r = t; r < NL; r += NT) {
    int lf = r / B, m = r % B, f = sm.fid[lf];
    int fr = a.free_rank[f];
    sL[r] = fr >= 0 ? a.lam_fwd[(int64_t)fr * B + m] : a.lamD[(int64_t)f * B + m];
    sLa[r] = fr >= 0 ? a.lam_adj[(int64_t)fr * B + m] : 0.0;
  }
  __syncthreads();
  for (int i = t; i < NU; i += NT) {
    double r = Fo[i];
    for (int c = 0; c < NL; ++c) r -= Bo[i * NL + c] * sL[c];
    sR[i] = r;
    double tt = 0.0;
    for (int c = 0; c < NL; ++c) tt += Co[c * NU + i] * sLa[c];
    sT[i] = tt;
  }
  __syncthreads();
  for (int i = t; i < NU; i += NT) {
    double u = 0.0, w = 0.0;
    for (int k = 0; k < NU; ++k) {
      u += Ai[i * NU + k] * sR[k];
      w -= Ai[k * NU + i] * sT[k];
    }
    sU[i] = u;
    sW[i] = w;
  }
  __syncthreads();
  if (a.dJdf_q)
    for (int q = t; q < NQ; q += NT) {
      double v = 0.0;
      for (int i = 0; i < NU; ++i) v += sW[i] * a.vol_phi[q * NU + i];
      a.dJdf_q[e * NQ + q] = a.vol_w[q] * sm.absdet * v;
    }
  double acc = 0.0;
  for (int i = t; i < NU; i += NT) {
    double v = 0.0;
    for (int j = 0; j < NU; ++j) v += sm.A[i * NU + j] * sU[j];
    for (int c = 0; c < NL; ++c) v += sm.Bm[i * NL + c] * sL[c];
    acc -= sW[i] * v;
  }
  for (int r = t; r < NL; r += NT) {
    double v = 0.0;
    for (int j = 0; j < NU; ++j) v += sm.Cm[r * NU + j] * sU[j];
    int lf = r / B, m = r % B;
    for (int n = 0; n < B; ++n) v += sm.Dd[lf * B * B + m * B + n] * sL[lf * B + n];
    acc -= sLa[r] * v;
  }
  sred[t] = acc;
  __syncthreads();
  if (t == 0) {
    double s2 = 0.0;
    for (int k = 0; k < NT; ++k) s2 += sred[k];
    a.dnu_elem[e] = s2;
  }
}

// ------------------------------------------------------------ dispatch
template <int D, int P>
static ah_status launch_element(const ElemArgs& a, hipStream_t st) {
  if (a.ne == 0) return AH_OK;
  using S = Sz<D, P>;
  // algorithmic bytes per element: cell, vertices, vertex velocity, facet
  // maps, source values in; condensed block, right-hand side and the kept
  // element blocks out
  const double per = (D + 1) * (4.0 + D * 8.0 + (D - 1) * 8.0 + 4.0 + D) + S::NQ * 8.0 +
                     (S::NL * S::NL + S::NL) * 8.0 +
                     (a.Ainv ? (S::NU * S::NU + 2.0 * S::NU * S::NL + S::NU) * 8.0 : 0.0);
  ProfScope ps;
  prof_begin(ps, "element", st, per * (double)a.ne);
  hipLaunchKernelGGL((k_element<D, P>), dim3(a.ne), dim3(64), 0, st, a);
  prof_end(ps);
  AH_LAUNCHED();
  return AH_OK;
}

static ah_status element_dispatch(int D, int p, const ElemArgs& a, hipStream_t st) {
  if (D == 2 && p == 1) return launch_element<2, 1>(a, st);
  if (D == 2 && p == 2) return launch_element<2, 2>(a, st);
  if (D == 2 && p == 3) return launch_element<2, 3>(a, st);
  if (D == 3 && p == 1) return launch_element<3, 1>(a, st);
  if (D == 3 && p == 2) return launch_element<3, 2>(a, st);
  if (D == 3 && p == 3) return launch_element<3, 3>(a, st);
  set_error("unsupported dim_st/p");
  return AH_EUNSUPPORTED;
}

template <int B>
static ah_status scale_to_csr(ah_system* s, const ah_mesh* m, hipStream_t st, int* d_err) {
  const int64_t nfree = s->nfree;
  const int64_t n = nfree * B;
  Arena& ar = s->arena;
  if (s->unscaled)
    hipLaunchKernelGGL(k_ident_blocks<B>, dim3(cdiv(std::max<int64_t>(nfree * B * B, 1), 256)), dim3(256), 0, st,
                       nfree, s->d_Dinv);
  else
    hipLaunchKernelGGL(k_diag_inv<B>, dim3(cdiv(std::max<int64_t>(nfree, 1), 64)), dim3(64), 0, st, nfree,
                       m->d_bsr_ptr, m->d_bsr_col, s->d_bval, s->d_Dinv, d_err);
  AH_LAUNCHED();
  const int64_t nob = (int64_t)m->odb_col.size();
  s->nnz = s->unscaled ? (int64_t)B * B * s->nnzb : n + (int64_t)B * B * nob;
  if (s->nnz >= ((int64_t)1 << 31)) {
    set_error("level-0 matrix has %lld entries (limit 2^31)", (long long)s->nnz);
    return AH_EUNSUPPORTED;
  }
  AH_TRY(ar.get(&s->d_rowptr, n + 1));
  AH_TRY(ar.get(&s->d_col, s->nnz));
  AH_TRY(ar.get(&s->d_val, s->nnz));
  if (!s->unscaled) AH_TRY(ar.get(&s->d_odv, nob * B * B));
  hipLaunchKernelGGL(k_scaled_rowptr<B>, dim3((unsigned)cdiv(n + 1, 256)), dim3(256), 0, st, nfree, m->d_bsr_ptr,
                     (const int64_t*)m->d_odb_ptr, (int)s->unscaled, s->d_rowptr);
  AH_LAUNCHED();
  const dim3 gw((unsigned)cdiv(std::max<int64_t>(nfree, 1) * 64, 256));
  hipLaunchKernelGGL(k_csr_scaled<B>, gw, dim3(256), 0, st, nfree, m->d_bsr_ptr, m->d_bsr_col, s->d_bval, s->d_Dinv,
                     s->d_col, s->d_val, (int)s->unscaled, (const int64_t*)m->d_odb_ptr, s->d_odv);
  AH_LAUNCHED();
  return AH_OK;
}

// H = H0 + Neumann term of g_q (NULL: none), then H_hat = D_b^-1 H.
template <int B>
static ah_status rhs_from_neumann(ah_system* s, const double* g_q, hipStream_t st) {
  const ah_mesh* m = s->mesh;
  const int64_t n = s->nfree * B;
  if (n == 0) return AH_OK;
  AH_HIP(hipMemcpyAsync(s->d_H, s->d_H0, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  const int64_t nbf = (int64_t)m->bfacets.size();
  if (g_q && nbf > 0) {
    hipLaunchKernelGGL(k_neumann<B>, dim3((unsigned)cdiv(nbf * B, 128)), dim3(128), 0, st, nbf, m->D, s->nqf,
                       m->d_bfacets, m->d_kind, m->d_free_rank, m->d_facet_vert, m->d_vert, s->tab.d_fac_w,
                       s->tab.d_fac_psi, g_q, s->d_H);
    AH_LAUNCHED();
  }
  hipLaunchKernelGGL(k_hhat<B>, dim3((unsigned)cdiv(n, 128)), dim3(128), 0, st, s->nfree, s->d_Dinv, s->d_H,
                     s->d_Hhat);
  AH_LAUNCHED();
  return AH_OK;
}

static ah_status rhs_dispatch(int b, ah_system* s, const double* g_q, hipStream_t st) {
  switch (b) {
    case 2: return rhs_from_neumann<2>(s, g_q, st);
    case 3: return rhs_from_neumann<3>(s, g_q, st);
    case 4: return rhs_from_neumann<4>(s, g_q, st);
    case 6: return rhs_from_neumann<6>(s, g_q, st);
    case 10: return rhs_from_neumann<10>(s, g_q, st);
  }
  set_error("unsupported facet block size %d", b);
  return AH_EUNSUPPORTED;
}

static ah_status scale_dispatch(int b, ah_system* s, const ah_mesh* m, hipStream_t st, int* d_err) {
  switch (b) {
    case 2: return scale_to_csr<2>(s, m, st, d_err);
    case 3: return scale_to_csr<3>(s, m, st, d_err);
    case 4: return scale_to_csr<4>(s, m, st, d_err);
    case 6: return scale_to_csr<6>(s, m, st, d_err);
    case 10: return scale_to_csr<10>(s, m, st, d_err);
  }
  set_error("unsupported facet block size %d", b);
  return AH_EUNSUPPORTED;
}

static void fill_common(ElemArgs& a, const ah_mesh* m, const RefTables& t) {
  a.ne = m->ne;
  a.vert = m->d_vert;
  a.cell = m->d_cell;
  a.elem_facet = m->d_elem_facet;
  a.facet_loc = m->d_facet_loc;
  a.kind = m->d_kind;
  a.bf_index = m->d_bf_index;
  a.free_rank = m->d_free_rank;
  a.elem_slot = m->d_elem_slot;
  a.vol_w = t.d_vol_w;
  a.vol_lam = t.d_vol_lam;
  a.vol_phi = t.d_vol_phi;
  a.vol_dphi = t.d_vol_dphi;
  a.fac_w = t.d_fac_w;
  a.fac_mu = t.d_fac_mu;
  a.fac_psi = t.d_fac_psi;
  a.fac_proj = t.d_fac_proj;
  a.ten_adv = t.d_ten_adv;
  a.ten_dif = t.d_ten_dif;
  for (int i = 0; i < 20; ++i)
    for (int c = 0; c < 3; ++c) a.mono[i][c] = (i < t.nu && c < t.D) ? (int8_t)t.mono[i * t.D + c] : 0;
}

template <int D, int P>
static ah_status launch_grad(const ElemArgs& a, hipStream_t st) {
  if (a.ne == 0) return AH_OK;
  hipLaunchKernelGGL((k_grad<D, P>), dim3(a.ne), dim3(64), 0, st, a);
  AH_LAUNCHED();
  return AH_OK;
}

ah_status grad_dispatch(const ah_system* s, const double* a_vert, const double* lam_fwd, const double* lam_adj,
                        double* dJdf_q, double* dnu_elem, hipStream_t st) {
  ElemArgs a{};
  fill_common(a, s->mesh, s->tab);
  a.a_vert = a_vert;
  a.nu = 1.0;
  a.alpha = s->alpha;
  a.lamD = s->d_lamD;
  a.Ainv = s->d_Ainv;
  a.Bm = s->d_Bm;
  a.Cm = s->d_Cm;
  a.Fv = s->d_Fv;
  a.lam_fwd = lam_fwd;
  a.lam_adj = lam_adj;
  a.dJdf_q = dJdf_q;
  a.dnu_elem = dnu_elem;
  int* err = nullptr;
  Arena tmp;
  tmp.stream = st;
  AH_TRY(tmp.get(&err, 1));
  a.err = err;
  ah_status rc;
  const int D = s->D, p = s->p;
  if (D == 2 && p == 1) rc = launch_grad<2, 1>(a, st);
  else if (D == 2 && p == 2) rc = launch_grad<2, 2>(a, st);
  else if (D == 2 && p == 3) rc = launch_grad<2, 3>(a, st);
  else if (D == 3 && p == 1) rc = launch_grad<3, 1>(a, st);
  else if (D == 3 && p == 2) rc = launch_grad<3, 2>(a, st);
  else if (D == 3 && p == 3) rc = launch_grad<3, 3>(a, st);
  else { set_error("unsupported dim_st/p"); rc = AH_EUNSUPPORTED; }
  tmp.release();
  return rc;
}

}  // namespace ah

using namespace ah;

extern "C" ah_status ah_quad_points(const ah_mesh* mc, int p, double* xq_elem, double* xq_bfacet, void* stream) {
  if (!mc) { set_error("null mesh"); return AH_EINVAL; }
  ah_mesh* m = const_cast<ah_mesh*>(mc);
  hipStream_t st = as_stream(stream);
  RefTables t;
  AH_TRY(build_ref_tables(m->D, p, t));
  Arena tmp;
  tmp.stream = st;
  AH_TRY(upload_ref_tables(t, tmp));
  double* d_vert = nullptr;
  int32_t *d_cell = nullptr, *d_bf = nullptr, *d_fv = nullptr;
  AH_TRY(tmp.get(&d_vert, m->vert.size()));
  AH_TRY(tmp.get(&d_cell, m->cell.size()));
  AH_TRY(tmp.get(&d_bf, m->bfacets.size()));
  AH_TRY(tmp.get(&d_fv, m->facet_vert.size()));
  AH_HIP(hipMemcpyAsync(d_vert, m->vert.data(), m->vert.size() * 8, hipMemcpyHostToDevice, st));
  AH_HIP(hipMemcpyAsync(d_cell, m->cell.data(), m->cell.size() * 4, hipMemcpyHostToDevice, st));
  AH_HIP(hipMemcpyAsync(d_bf, m->bfacets.data(), m->bfacets.size() * 4, hipMemcpyHostToDevice, st));
  AH_HIP(hipMemcpyAsync(d_fv, m->facet_vert.data(), m->facet_vert.size() * 4, hipMemcpyHostToDevice, st));
  if (xq_elem && m->ne) {
    hipLaunchKernelGGL(k_quad_points_elem, dim3(cdiv(m->ne * t.nq, 256)), dim3(256), 0, st, m->ne, m->D, t.nq, d_vert,
                       d_cell, t.d_vol_lam, xq_elem);
    AH_LAUNCHED();
  }
  if (xq_bfacet && m->nbf) {
    hipLaunchKernelGGL(k_quad_points_bfacet, dim3(cdiv(m->nbf * t.nqf, 256)), dim3(256), 0, st, m->nbf, m->D, t.nqf,
                       d_vert, d_bf, d_fv, t.d_fac_mu, xq_bfacet);
    AH_LAUNCHED();
  }
  AH_HIP(hipStreamSynchronize(st));
  tmp.release();
  return AH_OK;
}

static ah_status assemble_impl(const ah_mesh* mc, const ah_hdg_params* prm, double nu, const double* a_vert,
                               const double* a_qe, const double* a_qf, const double* f_q, const double* g_q,
                               void* stream, ah_system** out) {
  if (!(nu >= 0.0) || !std::isfinite(nu)) { set_error("hdg_assemble: nu must be finite and >= 0"); return AH_EINVAL; }
  if (!mc->bc_set) { set_error("hdg_assemble: boundary kinds not set"); return AH_EINVAL; }
  *out = nullptr;
  ah_mesh* m = const_cast<ah_mesh*>(mc);
  hipStream_t st = as_stream(stream);
  AH_TRY(mesh_upload(m, st));
  ah_system* s = new ah_system();
  s->arena.stream = st;
  s->mesh = m;
  s->D = m->D;
  s->p = prm->p;
  s->visc = nu;
  s->alpha = prm->alpha > 0.0 ? prm->alpha : 10.0 * prm->p * prm->p;
  s->keep = prm->keep_element_data != 0;
  s->unscaled = prm->no_block_scale != 0;
  auto fail = [&](ah_status code) { delete s; return code; };
  ah_status rc = build_ref_tables(m->D, prm->p, s->tab);
  if (rc) return fail(rc);
  if ((rc = upload_ref_tables(s->tab, s->arena))) return fail(rc);
  const RefTables& t = s->tab;
  s->nu = t.nu; s->b = t.b; s->nl = (m->D + 1) * t.b; s->nq = t.nq; s->nqf = t.nqf;
  s->nfree = m->nfree;
  s->n = m->nfree * t.b;
  s->nnzb = (int64_t)m->bsr_col.size();
  Arena& ar = s->arena;
  if ((rc = ar.get(&s->d_bval, s->nnzb * t.b * t.b))) return fail(rc);
  if ((rc = ar.get(&s->d_H, s->n))) return fail(rc);
  if ((rc = ar.get(&s->d_H0, s->n))) return fail(rc);
  if ((rc = ar.get(&s->d_Hhat, s->n))) return fail(rc);
  if ((rc = ar.get(&s->d_Dinv, s->nfree * t.b * t.b))) return fail(rc);
  if ((rc = ar.get(&s->d_lamD, m->nf * t.b))) return fail(rc);
  if (s->keep) {
    if ((rc = ar.get(&s->d_Ainv, m->ne * t.nu * t.nu))) return fail(rc);
    if ((rc = ar.get(&s->d_Bm, m->ne * t.nu * s->nl))) return fail(rc);
    if ((rc = ar.get(&s->d_Cm, m->ne * s->nl * t.nu))) return fail(rc);
    if ((rc = ar.get(&s->d_Fv, m->ne * t.nu))) return fail(rc);
  }
  int* d_err = nullptr;
  if ((rc = ar.get(&d_err, 1))) return fail(rc);
  if (hipMemsetAsync(d_err, 0, sizeof(int), st) != hipSuccess ||
      hipMemsetAsync(s->d_bval, 0, s->nnzb * t.b * t.b * sizeof(double), st) != hipSuccess ||
      hipMemsetAsync(s->d_H0, 0, s->n * sizeof(double), st) != hipSuccess ||
      hipMemsetAsync(s->d_lamD, 0, m->nf * t.b * sizeof(double), st) != hipSuccess) {
    set_error("hdg_assemble: memset failed");
    return fail(AH_EHIP);
  }
  ElemArgs a{};
  fill_common(a, m, t);
  a.a_vert = a_vert;
  a.a_qe = a_qe;
  a.a_qf = a_qf;
  a.f_q = f_q;
  a.g_q = g_q;
  a.nu = nu;
  a.alpha = s->alpha;
  a.bval = s->d_bval;
  a.H = s->d_H0;
  a.lamD = s->d_lamD;
  a.Ainv = s->d_Ainv;
  a.Bm = s->d_Bm;
  a.Cm = s->d_Cm;
  a.Fv = s->d_Fv;
  a.err = d_err;
  if ((rc = element_dispatch(m->D, prm->p, a, st))) return fail(rc);
  if ((rc = scale_dispatch(t.b, s, m, st, d_err))) return fail(rc);
  if ((rc = rhs_dispatch(t.b, s, g_q, st))) return fail(rc);
  int herr = 0;
  if ((rc = read_bytes(d_err, &herr, sizeof(int), st))) return fail(rc);
  if (herr) {
    set_error("hdg_assemble: singular %s", (herr & 4) ? "facet diagonal block (characteristic facet at nu = 0?)"
                                                      : (herr & 2) ? "element (degenerate cell)" : "element block A_K");
    return fail(AH_ESINGULAR);
  }
  *out = s;
  return AH_OK;
}

extern "C" ah_status ah_quad_points_facets(const ah_mesh* mc, int p, double* xq_facet, void* stream) {
  if (!mc || !xq_facet) { set_error("ah_quad_points_facets: null argument"); return AH_EINVAL; }
  ah_mesh* m = const_cast<ah_mesh*>(mc);
  if (m->nf == 0) return AH_OK;
  hipStream_t st = as_stream(stream);
  RefTables t;
  AH_TRY(build_ref_tables(m->D, p, t));
  Arena tmp;
  tmp.stream = st;
  AH_TRY(upload_ref_tables(t, tmp));
  std::vector<int32_t> ids((size_t)m->nf);
  for (int64_t f = 0; f < m->nf; ++f) ids[(size_t)f] = (int32_t)f;
  double* d_vert = nullptr;
  int32_t *d_ids = nullptr, *d_fv = nullptr;
  AH_TRY(tmp.get(&d_vert, m->vert.size()));
  AH_TRY(tmp.get(&d_ids, ids.size()));
  AH_TRY(tmp.get(&d_fv, m->facet_vert.size()));
  AH_HIP(hipMemcpyAsync(d_vert, m->vert.data(), m->vert.size() * 8, hipMemcpyHostToDevice, st));
  AH_HIP(hipMemcpyAsync(d_ids, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, st));
  AH_HIP(hipMemcpyAsync(d_fv, m->facet_vert.data(), m->facet_vert.size() * 4, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_quad_points_bfacet, dim3(cdiv(m->nf * t.nqf, 256)), dim3(256), 0, st, m->nf, m->D, t.nqf,
                     d_vert, d_ids, d_fv, t.d_fac_mu, xq_facet);
  AH_LAUNCHED();
  AH_HIP(hipStreamSynchronize(st));
  tmp.release();
  return AH_OK;
}

extern "C" ah_status hdg_assemble(const ah_mesh* mc, const ah_hdg_params* prm, double nu, const double* a_vert,
                                  const double* f_q, const double* g_q, void* stream, ah_system** out) {
  if (!mc || !prm || !out || !a_vert) { set_error("hdg_assemble: null argument"); return AH_EINVAL; }
  return assemble_impl(mc, prm, nu, a_vert, nullptr, nullptr, f_q, g_q, stream, out);
}

extern "C" ah_status hdg_assemble_q(const ah_mesh* mc, const ah_hdg_params* prm, double nu, const double* a_qe,
                                    const double* a_qf, const double* f_q, const double* g_q, void* stream,
                                    ah_system** out) {
  if (!mc || !prm || !out || !a_qe || !a_qf) { set_error("hdg_assemble_q: null argument"); return AH_EINVAL; }
  return assemble_impl(mc, prm, nu, nullptr, a_qe, a_qf, f_q, g_q, stream, out);
}

extern "C" ah_status hdg_update_neumann(ah_system* s, const double* g_q, void* stream) {
  if (!s) { set_error("hdg_update_neumann: null system"); return AH_EINVAL; }
  return rhs_dispatch(s->b, s, g_q, as_stream(stream));
}

extern "C" void ah_system_destroy(ah_system* s) { delete s; }

extern "C" ah_status ah_system_sizes(const ah_system* s, int64_t* n, int* b, int64_t* nnz) {
  if (!s) { set_error("null system"); return AH_EINVAL; }
  if (n) *n = s->n;
  if (b) *b = s->b;
  if (nnz) *nnz = s->nnz;
  return AH_OK;
}

extern "C" ah_status ah_system_export(const ah_system* s, int64_t* row_ptr, int32_t* col, double* val,
                                      double* h_hat, double* dinv, double* lam_dir, void* stream) {
  if (!s) { set_error("null system"); return AH_EINVAL; }
  hipStream_t st = as_stream(stream);
  if (row_ptr) AH_HIP(hipMemcpyAsync(row_ptr, s->d_rowptr, (s->n + 1) * 8, hipMemcpyDeviceToDevice, st));
  if (col) AH_HIP(hipMemcpyAsync(col, s->d_col, s->nnz * 4, hipMemcpyDeviceToDevice, st));
  if (val) AH_HIP(hipMemcpyAsync(val, s->d_val, s->nnz * 8, hipMemcpyDeviceToDevice, st));
  if (h_hat) AH_HIP(hipMemcpyAsync(h_hat, s->d_Hhat, s->n * 8, hipMemcpyDeviceToDevice, st));
  if (dinv) AH_HIP(hipMemcpyAsync(dinv, s->d_Dinv, s->nfree * s->b * s->b * 8, hipMemcpyDeviceToDevice, st));
  if (lam_dir) AH_HIP(hipMemcpyAsync(lam_dir, s->d_lamD, s->mesh->nf * s->b * 8, hipMemcpyDeviceToDevice, st));
  return AH_OK;
}
