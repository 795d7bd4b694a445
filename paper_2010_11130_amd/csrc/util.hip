// Device utilities: exclusive prefix sums used to turn per-row counts into
// CSR offsets.
#include <cstring>

#include "system.h"

namespace ah {

constexpr int SCAN_T = 256;
constexpr int SCAN_PER = 4;
constexpr int SCAN_TILE = SCAN_T * SCAN_PER;

template <class T>
__global__ __launch_bounds__(SCAN_T) void k_scan_tile(const T* __restrict__ in, int64_t* __restrict__ out,
                                                      int64_t* __restrict__ sums, int64_t n) {
  __shared__ int64_t s[SCAN_T];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_PER;
  int64_t v[SCAN_PER];
  int64_t tot = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? (int64_t)in[i] : 0;
    tot += v[k];
  }
  s[t] = tot;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int64_t x = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  int64_t run = s[t] - tot;   // exclusive prefix of this thread
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (t == SCAN_T - 1) sums[blockIdx.x] = s[t];
}

__global__ void k_scan_add(int64_t* __restrict__ out, const int64_t* __restrict__ offs, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / SCAN_TILE];
}

__global__ void k_scan_total(int64_t* out, const int64_t* sums_scanned, int64_t nb, int64_t n) {
  out[n] = sums_scanned[nb];
}

template <class T>
static ah_status scan_impl(const T* in, int64_t* out, int64_t n, hipStream_t st, Arena& tmp) {
  if (n == 0) {
    AH_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), st));
    return AH_OK;
  }
  int64_t nb = cdiv(n, SCAN_TILE);
  int64_t* sums = nullptr;
  AH_TRY(tmp.get(&sums, nb));
  hipLaunchKernelGGL(k_scan_tile<T>, dim3(nb), dim3(SCAN_T), 0, st, in, out, sums, n);
  AH_LAUNCHED();
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, out, sums, (int64_t)0, n);
    AH_LAUNCHED();
    return AH_OK;
  }
  int64_t* sums_sc = nullptr;
  AH_TRY(tmp.get(&sums_sc, nb + 1));
  AH_TRY(scan_impl<int64_t>(sums, sums_sc, nb, st, tmp));   // sums_sc[nb] = total
  hipLaunchKernelGGL(k_scan_add, dim3(cdiv(n, 256)), dim3(256), 0, st, out, sums_sc, n);
  AH_LAUNCHED();
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, out, sums_sc, nb, n);
  AH_LAUNCHED();
  return AH_OK;
}

ah_status scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t st, Arena& tmp) {
  return scan_impl<int64_t>(in, out, n, st, tmp);
}

ah_status scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t st, Arena& tmp) {
  return scan_impl<int32_t>(in, out, n, st, tmp);
}

ah_status read_i64(const int64_t* d, int64_t* h, hipStream_t st) {
  double* pin = pinned_scratch(1);
  if (!pin) { set_error("pinned host allocation failed"); return AH_ENOMEM; }
  AH_HIP(hipMemcpyAsync(pin, d, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  AH_HIP(hipStreamSynchronize(st));
  std::memcpy(h, pin, sizeof(int64_t));
  return AH_OK;
}

ah_status read_bytes(const void* d, void* h, size_t bytes, hipStream_t st) {
  double* pin = pinned_scratch((bytes + 7) / 8);
  if (!pin) { set_error("pinned host allocation failed"); return AH_ENOMEM; }
  AH_HIP(hipMemcpyAsync(pin, d, bytes, hipMemcpyDeviceToHost, st));
  AH_HIP(hipStreamSynchronize(st));
  std::memcpy(h, pin, bytes);
  return AH_OK;
}

}  // namespace ah
