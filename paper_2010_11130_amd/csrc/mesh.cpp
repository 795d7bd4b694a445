// Host side: error state, stream-ordered arena, quadrature rules, reference
// tables and mesh topology (facets as sorted vertex tuples, element-facet
// maps, free-facet block pattern, time-plane pairing).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <unordered_map>

#include "common.h"

namespace ah {

static thread_local std::string g_last_error = "no error";

const char* g_last_error_cstr() { return g_last_error.c_str(); }

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

// The library's caching device allocator (used unless the caller registers
// its own).  A freed block stays cached with its device and the stream it
// was freed on; a later request on the same device and stream takes the
// smallest cached block that holds it, if that block is at most twice the
// request, so the per-slab objects of a march and the solver workspaces of
// successive hierarchies reuse memory without new mappings.  Otherwise the
// memory comes from hipMalloc; when that runs out, the device is
// synchronized, every cached block of the device is released and the call
// is retried once.  Sizes are rounded up to 2 MiB.  Reuse on the freeing
// stream is safe in stream order: work enqueued after the free runs after
// the work that used the block before.
namespace {
constexpr size_t CACHE_ROUND = size_t(2) << 20;
std::mutex g_cache_mu;
std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void*>> g_cache;

// Frees every cached block of device dev (the caller has synchronized it).
void cache_release_device(int dev) {
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
      if (it->first.first == dev) {
        for (auto& b : it->second) drop.push_back(b.second);
        it = g_cache.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (void* q : drop) (void)hipFree(q);
}
}  // namespace

static hipError_t cache_alloc(void** p, size_t* bytes, hipStream_t st, int dev) {
  *bytes = (*bytes + CACHE_ROUND - 1) / CACHE_ROUND * CACHE_ROUND;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto c = g_cache.find({dev, st});
    if (c != g_cache.end()) {
      auto it = c->second.lower_bound(*bytes);
      if (it != c->second.end() && it->first <= 2 * *bytes) {
        *p = it->second;
        *bytes = it->first;
        c->second.erase(it);
        return hipSuccess;
      }
    }
  }
  hipError_t e = hipMalloc(p, *bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    cache_release_device(dev);
    e = hipMalloc(p, *bytes);
  }
  return e;
}

static void cache_free(void* p, size_t bytes, hipStream_t st, int dev) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  g_cache[{dev, st}].emplace(bytes, p);
}

// The caller's device allocator (ah_set_allocator), if one is registered.
static std::mutex g_alloc_mu;
static ah_alloc_fn g_alloc = nullptr;
static ah_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;

ah_status Arena::alloc(void** p, size_t bytes) {
  *p = nullptr;
  bytes = (std::max<size_t>(bytes, 16) + 255) & ~size_t(255);
  if (stream != cur_stream) left = 0;
  if (bytes > left) {
    size_t want = std::max(bytes, CHUNK);
    void* q = nullptr;
    ah_alloc_fn afn;
    ah_free_fn ffn;
    void* ctx;
    int dev = -1;
    {
      std::lock_guard<std::mutex> lock(g_alloc_mu);
      afn = g_alloc;
      ffn = g_free;
      ctx = g_alloc_ctx;
    }
    if (afn) {
      q = afn(ctx, (int64_t)want, (void*)stream);
      if (!q) {
        set_error("device allocation of %zu bytes failed (caller's allocator)", want);
        return AH_ENOMEM;
      }
    } else {
      ffn = nullptr;
      if (hipGetDevice(&dev) != hipSuccess) dev = 0;
      hipError_t e = cache_alloc(&q, &want, stream, dev);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
        return AH_ENOMEM;
      }
    }
    ptrs.push_back({q, stream, want, ffn, ctx, dev});
    if (want > CHUNK) {          // dedicated chunk for a large buffer
      *p = q;
      return AH_OK;
    }
    cur = static_cast<char*>(q);
    left = want;
    cur_stream = stream;
  }
  *p = cur;
  cur += bytes;
  left -= bytes;
  return AH_OK;
}

void Arena::release() {
  for (auto& c : ptrs) {
    if (c.free_fn)
      c.free_fn(c.ctx, c.p, (int64_t)c.bytes, (void*)c.stream);
    else
      cache_free(c.p, c.bytes, c.stream, c.dev);
  }
  ptrs.clear();
  cur = nullptr;
  left = 0;
}

double* pinned_scratch(size_t doubles) {
  static thread_local double* buf = nullptr;
  static thread_local size_t cap = 0;
  if (doubles > cap) {
    size_t want = std::max<size_t>(doubles, 8192);
    double* nb = nullptr;
    if (hipHostMalloc((void**)&nb, want * sizeof(double), hipHostMallocDefault) != hipSuccess) return nullptr;
    // the previous buffer is kept: a caller may still hold it
    buf = nb;
    cap = want;
  }
  return buf;
}

// ------------------------------------------------------------ quadrature
// Jacobi polynomial P_n^(a,0)(x) and its derivative by the three-term
// recurrence; derivative from d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1).
static void jacobi_pd(int n, double a, double b, double x, double* pv, double* dv) {
  auto P = [](int n, double a, double b, double x) {
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = 0.5 * ((a - b) + (a + b + 2.0) * x);
    for (int k = 1; k < n; ++k) {
      double c = 2.0 * k + a + b;
      double a1 = 2.0 * (k + 1) * (k + a + b + 1) * c;
      double a2 = (c + 1) * (a * a - b * b);
      double a3 = c * (c + 1) * (c + 2);
      double a4 = 2.0 * (k + a) * (k + b) * (c + 2);
      double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
      p0 = p1;
      p1 = p2;
    }
    return p1;
  };
  *pv = P(n, a, b, x);
  *dv = n == 0 ? 0.0 : 0.5 * (n + a + b + 1) * P(n - 1, a + 1, b + 1, x);
}

// Gauss rule on [0,1] for the weight (1-s)^alpha: Newton on the zeros of
// P_n^(alpha,0) with deflation of the roots already found.
void gauss_jacobi01(int n, double alpha, double* s, double* w) {
  std::vector<double> r(n);
  for (int k = 0; k < n; ++k) {
    double x = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
    if (k > 0) x = 0.5 * (x + r[k - 1]);
    for (int it = 0; it < 100; ++it) {
      double pv, dv;
      jacobi_pd(n, alpha, 0.0, x, &pv, &dv);
      double sdef = 0.0;
      for (int j = 0; j < k; ++j) sdef += 1.0 / (x - r[j]);
      double dx = pv / (dv - sdef * pv);
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    r[k] = x;
  }
  std::sort(r.begin(), r.end());
  for (int k = 0; k < n; ++k) {
    double pv, dv;
    jacobi_pd(n, alpha, 0.0, r[k], &pv, &dv);
    double wy = std::pow(2.0, alpha + 1.0) / ((1.0 - r[k] * r[k]) * dv * dv);
    s[k] = 0.5 * (1.0 + r[k]);
    w[k] = wy / std::pow(2.0, alpha + 1.0);
  }
}

// Conical-product rule on the reference dim-simplex, s_1 fastest.
void simplex_rule(int dim, int n, std::vector<double>& xi, std::vector<double>& w) {
  if (dim == 0) {
    xi.assign(0, 0.0);
    w.assign(1, 1.0);
    return;
  }
  std::vector<std::vector<double>> S(dim, std::vector<double>(n)), W(dim, std::vector<double>(n));
  for (int k = 0; k < dim; ++k) gauss_jacobi01(n, (double)k, S[k].data(), W[k].data());
  int nq = 1;
  for (int k = 0; k < dim; ++k) nq *= n;
  xi.assign((size_t)nq * dim, 0.0);
  w.assign(nq, 0.0);
  for (int q = 0; q < nq; ++q) {
    int i[3] = {0, 0, 0};
    int t = q;
    for (int k = 0; k < dim; ++k) { i[k] = t % n; t /= n; }
    double s1 = S[0][i[0]], s2 = dim > 1 ? S[1][i[1]] : 0.0, s3 = dim > 2 ? S[2][i[2]] : 0.0;
    double ww = W[0][i[0]] * (dim > 1 ? W[1][i[1]] : 1.0) * (dim > 2 ? W[2][i[2]] : 1.0);
    if (dim == 1) {
      xi[q] = s1;
    } else if (dim == 2) {
      xi[q * 2 + 0] = s1 * (1.0 - s2);
      xi[q * 2 + 1] = s2;
    } else {
      xi[q * 3 + 0] = s1 * (1.0 - s2) * (1.0 - s3);
      xi[q * 3 + 1] = s2 * (1.0 - s3);
      xi[q * 3 + 2] = s3;
    }
    w[q] = ww;
  }
}

void lattice(int dim, int p, std::vector<int>& idx) {
  idx.clear();
  if (dim == 0) return;
  int i[3];
  int n = p + 1;
  int tot = 1;
  for (int k = 0; k < dim; ++k) tot *= n;
  for (int q = 0; q < tot; ++q) {   // i_1 fastest
    int t = q, s = 0;
    for (int k = 0; k < dim; ++k) { i[k] = t % n; t /= n; s += i[k]; }
    if (s <= p)
      for (int k = 0; k < dim; ++k) idx.push_back(i[k]);
  }
}

// Lagrange product basis on a simplex at barycentric coordinates lam[dim+1].
static double lagr(int dim, int p, const int* beta, const double* lam) {
  double v = 1.0;
  for (int k = 0; k <= dim; ++k)
    for (int m = 0; m < beta[k]; ++m) v *= (p * lam[k] - m) / (m + 1.0);
  return v;
}

static bool invert_small(int n, std::vector<double>& A) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    for (int j = 0; j < n; ++j) { std::swap(A[c * n + j], A[piv * n + j]); std::swap(I[c * n + j], I[piv * n + j]); }
    double d = A[c * n + c];
    for (int j = 0; j < n; ++j) { A[c * n + j] /= d; I[c * n + j] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { A[r * n + j] -= f * A[c * n + j]; I[r * n + j] -= f * I[c * n + j]; }
    }
  }
  A = I;
  return true;
}

ah_status build_ref_tables(int D, int p, RefTables& t) {
  if (D < 2 || D > 3 || p < 1 || p > 3) {
    set_error("unsupported dim_st=%d p=%d (dim_st in 2..3, p in 1..3)", D, p);
    return AH_EUNSUPPORTED;
  }
  t.D = D; t.p = p;
  t.nu = dim_p(D, p);
  t.b = dim_p(D - 1, p);
  int n1 = p + 2;
  std::vector<double> xi, w;
  simplex_rule(D, n1, xi, w);
  t.nq = (int)w.size();
  t.vol_w = w;
  t.vol_lam.assign((size_t)t.nq * (D + 1), 0.0);
  // element basis: monomials xi^alpha, |alpha| <= p, ordered like the lattice
  std::vector<int> mono;
  lattice(D, p, mono);
  t.mono = mono;
  t.vol_phi.assign((size_t)t.nq * t.nu, 0.0);
  t.vol_dphi.assign((size_t)t.nq * t.nu * D, 0.0);
  for (int q = 0; q < t.nq; ++q) {
    double s = 0;
    for (int a = 0; a < D; ++a) { t.vol_lam[q * (D + 1) + a + 1] = xi[q * D + a]; s += xi[q * D + a]; }
    t.vol_lam[q * (D + 1)] = 1.0 - s;
    for (int i = 0; i < t.nu; ++i) {
      const int* al = &mono[i * D];
      double v = 1.0;
      for (int a = 0; a < D; ++a) v *= std::pow(xi[q * D + a], al[a]);
      t.vol_phi[q * t.nu + i] = v;
      for (int a = 0; a < D; ++a) {
        double d = 0.0;
        if (al[a] > 0) {
          d = al[a];
          for (int c = 0; c < D; ++c)
            d *= std::pow(xi[q * D + c], c == a ? al[c] - 1 : al[c]);
        }
        t.vol_dphi[((size_t)q * t.nu + i) * D + a] = d;
      }
    }
  }
  // facet rule and Lagrange facet basis (vertex order = sorted global ids)
  std::vector<double> xf, wf;
  simplex_rule(D - 1, n1, xf, wf);
  t.nqf = (int)wf.size();
  double fact = 1.0;
  for (int k = 2; k <= D - 1; ++k) fact *= k;
  t.fac_w.resize(t.nqf);
  t.fac_mu.assign((size_t)t.nqf * D, 0.0);
  for (int q = 0; q < t.nqf; ++q) {
    t.fac_w[q] = wf[q] * fact;
    double s = 0;
    for (int a = 0; a < D - 1; ++a) { t.fac_mu[q * D + a + 1] = xf[q * (D - 1) + a]; s += xf[q * (D - 1) + a]; }
    t.fac_mu[q * D] = 1.0 - s;
  }
  std::vector<int> flat;
  lattice(D - 1, p, flat);
  t.fac_psi.assign((size_t)t.nqf * t.b, 0.0);
  for (int m = 0; m < t.b; ++m) {
    int beta[3] = {p, 0, 0};
    for (int a = 0; a < D - 1; ++a) { beta[a + 1] = flat[m * (D - 1) + a]; beta[0] -= beta[a + 1]; }
    for (int q = 0; q < t.nqf; ++q) t.fac_psi[q * t.b + m] = lagr(D - 1, p, beta, &t.fac_mu[q * D]);
  }
  std::vector<double> M((size_t)t.b * t.b, 0.0);
  for (int q = 0; q < t.nqf; ++q)
    for (int m = 0; m < t.b; ++m)
      for (int k = 0; k < t.b; ++k) M[m * t.b + k] += t.fac_w[q] * t.fac_psi[q * t.b + m] * t.fac_psi[q * t.b + k];
  if (!invert_small(t.b, M)) { set_error("singular facet mass matrix"); return AH_EINVAL; }
  t.fac_proj.assign((size_t)t.b * t.nqf, 0.0);
  for (int m = 0; m < t.b; ++m)
    for (int q = 0; q < t.nqf; ++q) {
      double v = 0;
      for (int k = 0; k < t.b; ++k) v += M[m * t.b + k] * t.fac_psi[q * t.b + k] * t.fac_w[q];
      t.fac_proj[m * t.nqf + q] = v;
    }
  // reference tensors of the volume terms
  {
    const int nu = t.nu, nn = nu * nu;
    t.ten_adv.assign((size_t)(D + 1) * D * nn, 0.0);
    t.ten_dif.assign((size_t)D * D * nn, 0.0);
    for (int q = 0; q < t.nq; ++q) {
      const double wq = t.vol_w[q];
      const double* ph = &t.vol_phi[(size_t)q * nu];
      const double* dp = &t.vol_dphi[(size_t)q * nu * D];
      for (int i = 0; i < nu; ++i)
        for (int j = 0; j < nu; ++j) {
          for (int r = 0; r < D; ++r) {
            const double gi = wq * dp[i * D + r] * ph[j];
            for (int k = 0; k <= D; ++k)
              t.ten_adv[((size_t)(k * D + r) * nn) + i * nu + j] += t.vol_lam[q * (D + 1) + k] * gi;
            for (int s2 = 0; s2 < D; ++s2)
              t.ten_dif[((size_t)(r * D + s2) * nn) + i * nu + j] += wq * dp[j * D + r] * dp[i * D + s2];
          }
        }
    }
  }
  // monomial basis at the element lattice nodes
  std::vector<int> elat;
  lattice(D, p, elat);
  t.lat_phi.assign((size_t)t.nu * t.nu, 0.0);
  for (int k = 0; k < t.nu; ++k)
    for (int i = 0; i < t.nu; ++i) {
      double v = 1.0;
      for (int a = 0; a < D; ++a) v *= std::pow((double)elat[k * D + a] / p, mono[i * D + a]);
      t.lat_phi[k * t.nu + i] = v;
    }
  return AH_OK;
}

static ah_status upload(Arena& ar, const std::vector<double>& h, double** d) {
  AH_TRY(ar.get(d, h.size()));
  AH_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, ar.stream));
  return AH_OK;
}

ah_status upload_ref_tables(RefTables& t, Arena& ar) {
  AH_TRY(upload(ar, t.vol_w, &t.d_vol_w));
  AH_TRY(upload(ar, t.vol_lam, &t.d_vol_lam));
  AH_TRY(upload(ar, t.vol_phi, &t.d_vol_phi));
  AH_TRY(upload(ar, t.vol_dphi, &t.d_vol_dphi));
  AH_TRY(upload(ar, t.fac_w, &t.d_fac_w));
  AH_TRY(upload(ar, t.fac_mu, &t.d_fac_mu));
  AH_TRY(upload(ar, t.fac_psi, &t.d_fac_psi));
  AH_TRY(upload(ar, t.fac_proj, &t.d_fac_proj));
  AH_TRY(upload(ar, t.lat_phi, &t.d_lat_phi));
  AH_TRY(upload(ar, t.ten_adv, &t.d_ten_adv));
  AH_TRY(upload(ar, t.ten_dif, &t.d_ten_dif));
  return AH_OK;
}

}  // namespace ah

using namespace ah;

// ------------------------------------------------------------------ mesh
static double det_small(int D, const double* J) {
  if (D == 2) return J[0] * J[3] - J[1] * J[2];
  return J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
         J[2] * (J[3] * J[7] - J[4] * J[6]);
}

extern "C" ah_status ah_mesh_create(int D, int64_t nv, const double* vert, int64_t ne,
                                    const int32_t* cell, ah_mesh** out) {
  if (!out || !vert || !cell || nv <= 0 || ne <= 0 || D < 2 || D > 3) {
    set_error("ah_mesh_create: invalid arguments");
    return AH_EINVAL;
  }
  if (ne * (D + 1) >= (int64_t)1 << 31 || nv >= (int64_t)1 << 31) {
    set_error("ah_mesh_create: mesh too large for 32-bit indices");
    return AH_EUNSUPPORTED;
  }
  *out = nullptr;
  ah_mesh* m = new ah_mesh();
  m->D = D; m->nv = nv; m->ne = ne;
  m->vert.assign(vert, vert + nv * D);
  m->cell.assign(cell, cell + ne * (D + 1));
  for (int64_t i = 0; i < ne * (D + 1); ++i)
    if (cell[i] < 0 || cell[i] >= nv) {
      delete m;
      set_error("ah_mesh_create: vertex id out of range in cell %lld", (long long)(i / (D + 1)));
      return AH_EINVAL;
    }
  for (int64_t e = 0; e < ne; ++e) {
    double J[9];
    const int32_t* c = &cell[e * (D + 1)];
    for (int r = 0; r < D; ++r)
      for (int a = 0; a < D; ++a) J[r * D + a] = vert[(int64_t)c[a + 1] * D + r] - vert[(int64_t)c[0] * D + r];
    double dj = det_small(D, J);
    if (!(std::fabs(dj) > 0.0) || !std::isfinite(dj)) {
      delete m;
      set_error("ah_mesh_create: degenerate cell %lld", (long long)e);
      return AH_ESINGULAR;
    }
  }
  // local facets: sorted vertex tuples
  struct LF { int32_t v[3]; int64_t id; };
  int64_t nl = ne * (D + 1);
  std::vector<LF> lf(nl);
  m->facet_loc.assign(nl * D, 0);
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t* c = &m->cell[e * (D + 1)];
    for (int f = 0; f <= D; ++f) {
      int loc[3], k = 0;
      for (int a = 0; a <= D; ++a)
        if (a != f) loc[k++] = a;
      // stable sort of local indices by global id
      std::sort(loc, loc + D, [&](int x, int y) { return c[x] < c[y] || (c[x] == c[y] && x < y); });
      LF& t = lf[e * (D + 1) + f];
      t.v[2] = -1;
      for (int s = 0; s < D; ++s) { t.v[s] = c[loc[s]]; m->facet_loc[(e * (D + 1) + f) * D + s] = (uint8_t)loc[s]; }
      t.id = e * (D + 1) + f;
    }
  }
  std::vector<int64_t> order(nl);
  std::iota(order.begin(), order.end(), 0);
  auto less = [&](int64_t a, int64_t b) {
    const LF& x = lf[a];
    const LF& y = lf[b];
    for (int s = 0; s < D; ++s)
      if (x.v[s] != y.v[s]) return x.v[s] < y.v[s];
    return a < b;
  };
  std::sort(order.begin(), order.end(), less);
  m->elem_facet.assign(nl, -1);
  m->facet_vert.clear();
  m->facet_elem.clear();
  int64_t nf = 0;
  for (int64_t k = 0; k < nl; ++k) {
    const LF& x = lf[order[k]];
    bool same = k > 0;
    if (same) {
      const LF& y = lf[order[k - 1]];
      for (int s = 0; s < D; ++s) same = same && x.v[s] == y.v[s];
    }
    if (!same) {
      for (int s = 0; s < D; ++s) m->facet_vert.push_back(x.v[s]);
      m->facet_elem.push_back((int32_t)(x.id / (D + 1)));
      m->facet_elem.push_back(-1);
      ++nf;
    } else {
      int32_t* fe = &m->facet_elem[(nf - 1) * 2];
      if (fe[1] != -1) {
        delete m;
        set_error("ah_mesh_create: facet shared by more than two cells");
        return AH_EINVAL;
      }
      fe[1] = (int32_t)(x.id / (D + 1));
    }
    m->elem_facet[x.id] = (int32_t)(nf - 1);
  }
  m->nf = nf;
  m->bf_index.assign(nf, -1);
  for (int64_t f = 0; f < nf; ++f)
    if (m->facet_elem[2 * f + 1] < 0) {
      m->bf_index[f] = (int32_t)m->bfacets.size();
      m->bfacets.push_back((int32_t)f);
    }
  m->nbf = (int64_t)m->bfacets.size();
  m->kind.assign(nf, 0);
  // time planes and the pairing of initial-plane with final-plane facets
  m->t_min = 1e300; m->t_max = -1e300;
  for (int64_t v = 0; v < nv; ++v) {
    m->t_min = std::min(m->t_min, m->vert[v * D]);
    m->t_max = std::max(m->t_max, m->vert[v * D]);
  }
  *out = m;
  return AH_OK;
}

ah_mesh::~ah_mesh() {
  void* ptrs[] = {d_vert, d_cell, d_elem_facet, d_facet_loc, d_kind, d_bf_index, d_bfacets,
                  d_facet_vert, d_free_rank, d_elem_slot, d_bsr_ptr, d_bsr_col, d_odb_ptr, d_odb_col,
                  d_pair, d_pair_perm};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

extern "C" void ah_mesh_destroy(ah_mesh* m) { delete m; }

namespace ah {
template <class T>
static ah_status up(T** d, const std::vector<T>& h, hipStream_t st) {
  if (*d) { (void)hipFree(*d); *d = nullptr; }
  size_t bytes = std::max<size_t>(h.size() * sizeof(T), 16);
  hipError_t e = hipMalloc((void**)d, bytes);
  if (e != hipSuccess) { set_error("hipMalloc(%zu): %s", bytes, hipGetErrorString(e)); return AH_ENOMEM; }
  if (!h.empty()) AH_HIP(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return AH_OK;
}

// Upload the topology once (after the boundary kinds are set).
ah_status mesh_upload(ah_mesh* m, hipStream_t st) {
  std::lock_guard<std::mutex> lock(m->lazy_mu);
  if (m->dev_ready) return AH_OK;
  AH_TRY(up(&m->d_vert, m->vert, st));
  AH_TRY(up(&m->d_cell, m->cell, st));
  AH_TRY(up(&m->d_elem_facet, m->elem_facet, st));
  AH_TRY(up(&m->d_facet_loc, m->facet_loc, st));
  AH_TRY(up(&m->d_kind, m->kind, st));
  AH_TRY(up(&m->d_bf_index, m->bf_index, st));
  AH_TRY(up(&m->d_bfacets, m->bfacets, st));
  AH_TRY(up(&m->d_facet_vert, m->facet_vert, st));
  AH_TRY(up(&m->d_free_rank, m->free_rank, st));
  AH_TRY(up(&m->d_elem_slot, m->elem_slot, st));
  AH_TRY(up(&m->d_bsr_ptr, m->bsr_ptr, st));
  AH_TRY(up(&m->d_bsr_col, m->bsr_col, st));
  AH_TRY(up(&m->d_odb_ptr, m->odb_ptr, st));
  AH_TRY(up(&m->d_odb_col, m->odb_col, st));
  AH_HIP(hipStreamSynchronize(st));
  m->dev_ready = true;
  return AH_OK;
}

// Pair this mesh's initial-plane boundary facets with src's final-plane
// facets having the same spatial vertex coordinates.
ah_status mesh_pair_time_planes(ah_mesh* m, const ah_mesh* src, hipStream_t st) {
  std::lock_guard<std::mutex> lock(m->lazy_mu);
  if (m->pair_src == src && m->d_pair) return AH_OK;
  const int D = m->D;
  auto on_plane = [](const ah_mesh* mm, int64_t f, double t) {
    for (int s = 0; s < mm->D; ++s)
      if (std::fabs(mm->vert[(int64_t)mm->facet_vert[f * mm->D + s] * mm->D] - t) > 1e-12) return false;
    return true;
  };
  auto key_of = [](const ah_mesh* mm, int64_t f, std::vector<std::pair<std::vector<long long>, int>>& pts) {
    pts.clear();
    for (int s = 0; s < mm->D; ++s) {
      std::vector<long long> k;
      for (int c = 1; c < mm->D; ++c)
        k.push_back(llround(mm->vert[(int64_t)mm->facet_vert[f * mm->D + s] * mm->D + c] * 1e10));
      pts.push_back({k, s});
    }
    std::sort(pts.begin(), pts.end());
  };
  std::map<std::vector<long long>, std::pair<int32_t, std::vector<int>>> tops;
  std::vector<std::pair<std::vector<long long>, int>> pts;
  for (int64_t k = 0; k < src->nbf; ++k) {
    int64_t f = src->bfacets[k];
    if (!on_plane(src, f, src->t_max)) continue;
    key_of(src, f, pts);
    std::vector<long long> key;
    std::vector<int> ord;
    for (auto& pr : pts) { key.insert(key.end(), pr.first.begin(), pr.first.end()); ord.push_back(pr.second); }
    tops[key] = {(int32_t)f, ord};
  }
  std::vector<int32_t> pair;
  std::vector<uint8_t> perm;
  for (int64_t k = 0; k < m->nbf; ++k) {
    int64_t f = m->bfacets[k];
    if (!on_plane(m, f, m->t_min)) continue;
    key_of(m, f, pts);
    std::vector<long long> key;
    std::vector<int> ord;
    for (auto& pr : pts) { key.insert(key.end(), pr.first.begin(), pr.first.end()); ord.push_back(pr.second); }
    auto it = tops.find(key);
    if (it == tops.end()) continue;
    pair.push_back((int32_t)k);
    pair.push_back(it->second.first);
    // our sorted vertex ord[r] sits where src's sorted vertex it->second.second[r] sits
    std::vector<uint8_t> pm(D, 0);
    for (int r = 0; r < D; ++r) pm[ord[r]] = (uint8_t)it->second.second[r];
    perm.insert(perm.end(), pm.begin(), pm.end());
  }
  m->npair = (int64_t)pair.size() / 2;
  AH_TRY(up(&m->d_pair, pair, st));
  AH_TRY(up(&m->d_pair_perm, perm, st));
  AH_HIP(hipStreamSynchronize(st));
  m->pair_src = src;
  return AH_OK;
}
}  // namespace ah

extern "C" ah_status ah_mesh_sizes(const ah_mesh* m, int64_t* nf, int64_t* nbf) {
  if (!m) { set_error("null mesh"); return AH_EINVAL; }
  if (nf) *nf = m->nf;
  if (nbf) *nbf = m->nbf;
  return AH_OK;
}

extern "C" ah_status ah_mesh_facets(const ah_mesh* m, int32_t* fv, int32_t* fe) {
  if (!m) { set_error("null mesh"); return AH_EINVAL; }
  if (fv) std::memcpy(fv, m->facet_vert.data(), m->facet_vert.size() * sizeof(int32_t));
  if (fe) std::memcpy(fe, m->facet_elem.data(), m->facet_elem.size() * sizeof(int32_t));
  return AH_OK;
}

extern "C" ah_status ah_mesh_boundary_facets(const ah_mesh* m, int32_t* ids) {
  if (!m || !ids) { set_error("null argument"); return AH_EINVAL; }
  std::memcpy(ids, m->bfacets.data(), m->bfacets.size() * sizeof(int32_t));
  return AH_OK;
}

extern "C" ah_status ah_mesh_set_bc(ah_mesh* m, const int8_t* kind) {
  if (!m || !kind) { set_error("null argument"); return AH_EINVAL; }
  const int D = m->D;
  for (int64_t f = 0; f < m->nf; ++f) {
    bool bdry = m->facet_elem[2 * f + 1] < 0;
    if ((!bdry && kind[f] != 0) || (bdry && kind[f] != 1 && kind[f] != 2)) {
      set_error("ah_mesh_set_bc: facet %lld: kind %d invalid for a%s facet", (long long)f, (int)kind[f],
                bdry ? " boundary" : "n interior");
      return AH_EINVAL;
    }
  }
  m->kind.assign(kind, kind + m->nf);
  m->dev_ready = false;
  m->free_rank.assign(m->nf, -1);
  int64_t nfree = 0;
  for (int64_t f = 0; f < m->nf; ++f)
    if (kind[f] != 1) m->free_rank[f] = (int32_t)nfree++;
  m->nfree = nfree;
  // block pattern of the free facets: facets sharing a cell
  m->bsr_ptr.assign(nfree + 1, 0);
  m->bsr_col.clear();
  std::vector<int32_t> tmp;
  for (int64_t f = 0; f < m->nf; ++f) {
    if (m->free_rank[f] < 0) continue;
    tmp.clear();
    for (int s = 0; s < 2; ++s) {
      int32_t e = m->facet_elem[2 * f + s];
      if (e < 0) continue;
      for (int k = 0; k <= D; ++k) {
        int32_t g = m->elem_facet[(int64_t)e * (D + 1) + k];
        if (m->free_rank[g] >= 0) tmp.push_back(m->free_rank[g]);
      }
    }
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    for (int32_t c : tmp) m->bsr_col.push_back(c);
    m->bsr_ptr[m->free_rank[f] + 1] = (int64_t)m->bsr_col.size();
  }
  // off-diagonal blocks only (every free facet couples to itself once)
  m->odb_ptr.assign(nfree + 1, 0);
  m->odb_col.clear();
  m->odb_col.reserve(m->bsr_col.size() - (size_t)nfree);
  for (int64_t r = 0; r < nfree; ++r) {
    for (int64_t k = m->bsr_ptr[r]; k < m->bsr_ptr[r + 1]; ++k)
      if (m->bsr_col[k] != r) m->odb_col.push_back(m->bsr_col[k]);
    m->odb_ptr[r + 1] = (int64_t)m->odb_col.size();
  }
  const int nb = (D + 1) * (D + 1);
  m->elem_slot.assign(m->ne * nb, -1);
  for (int64_t e = 0; e < m->ne; ++e)
    for (int i = 0; i <= D; ++i) {
      int32_t ri = m->free_rank[m->elem_facet[e * (D + 1) + i]];
      if (ri < 0) continue;
      for (int j = 0; j <= D; ++j) {
        int32_t rj = m->free_rank[m->elem_facet[e * (D + 1) + j]];
        if (rj < 0) continue;
        const int32_t* b0 = &m->bsr_col[m->bsr_ptr[ri]];
        const int32_t* b1 = &m->bsr_col[m->bsr_ptr[ri + 1]];
        const int32_t* it = std::lower_bound(b0, b1, rj);
        m->elem_slot[e * nb + i * (D + 1) + j] = (int32_t)(m->bsr_ptr[ri] + (it - b0));
      }
    }
  m->bc_set = true;
  return AH_OK;
}

extern "C" ah_status ah_sizes(int D, int p, int* nq, int* nqf, int* nu, int* b) {
  if (D < 2 || D > 3 || p < 1 || p > 3) { set_error("unsupported dim_st/p"); return AH_EUNSUPPORTED; }
  int n1 = p + 2;
  if (nq) *nq = D == 2 ? n1 * n1 : n1 * n1 * n1;
  if (nqf) *nqf = D == 2 ? n1 : n1 * n1;
  if (nu) *nu = dim_p(D, p);
  if (b) *b = dim_p(D - 1, p);
  return AH_OK;
}

extern "C" ah_status ah_quad_rule(int dim, int n, double* xi, double* w) {
  if (dim < 0 || dim > 3 || n < 1 || n > 32 || !w) { set_error("ah_quad_rule: invalid arguments"); return AH_EINVAL; }
  std::vector<double> x, ww;
  simplex_rule(dim, n, x, ww);
  if (xi && !x.empty()) std::memcpy(xi, x.data(), x.size() * sizeof(double));
  std::memcpy(w, ww.data(), ww.size() * sizeof(double));
  return AH_OK;
}

extern "C" const char* ah_last_error(void) { return ah::g_last_error_cstr(); }

extern "C" ah_status ah_pool_trim(void) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    ah::set_error("ah_pool_trim: %s", hipGetErrorString(e));
    return AH_EHIP;
  }
  cache_release_device(dev);
  return AH_OK;
}

extern "C" ah_status ah_set_allocator(ah_alloc_fn alloc, ah_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    ah::set_error("ah_set_allocator: alloc and free must both be set or both be NULL");
    return AH_EINVAL;
  }
  std::lock_guard<std::mutex> lock(ah::g_alloc_mu);
  ah::g_alloc = alloc;
  ah::g_free = free_fn;
  ah::g_alloc_ctx = alloc ? ctx : nullptr;
  return AH_OK;
}
