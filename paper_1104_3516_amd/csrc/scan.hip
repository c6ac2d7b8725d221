// scan.hip - exclusive prefix sum of int32 counts (out has n+1 entries,
// out[n] = total).  Three passes: per-block totals, a single-block scan of
// the totals, and the per-block scan with its offset added.
#include "cd_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;

// inclusive scan of one value per thread across the block; returns the
// inclusive prefix and writes the block total to *total
__device__ int block_inclusive_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave-level inclusive scan with shuffles
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int k = 0; k < kThreads / 64; ++k) {
      int s = sh[k];
      sh[k] = acc;
      acc += s;
    }
    sh[kThreads / 64] = acc;
  }
  __syncthreads();
  v += sh[wave];
  *total = sh[kThreads / 64];
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(kThreads) void k_block_sums(const int* in, int64_t n, int* sums) {
  __shared__ int sh[kThreads / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * kTile;
  int s = 0;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  int total;
  block_inclusive_scan(s, sh, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_sums(int* sums, int nb, int* grand) {
  __shared__ int sh[kThreads / 64 + 1];
  int carry = 0;
  for (int base = 0; base < nb; base += kThreads) {
    int i = base + threadIdx.x;
    int v = i < nb ? sums[i] : 0;
    int total;
    int inc = block_inclusive_scan(v, sh, &total);
    if (i < nb) sums[i] = carry + inc - v;
    carry += total;
  }
  if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_tiles(const int* in, int* out, int64_t n,
                                                        const int* sums) {
  __shared__ int sh[kThreads / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int vals[kItems];
  int s = 0;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    vals[k] = i < n ? in[i] : 0;
    s += vals[k];
  }
  int total;
  int inc = block_inclusive_scan(s, sh, &total);
  int run = sums[blockIdx.x] + inc - s;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += vals[k];
  }
}

}  // namespace

hipError_t cd_scan_exclusive(cd_ctx* c, const int* in, int* out, int64_t n) {
  int nb = (int)((n + kTile - 1) / kTile);
  if (nb < 1) nb = 1;
  if (c->scan_tmp_cap < nb) {
    if (c->scan_tmp) (void)hipFree(c->scan_tmp);
    c->scan_tmp = nullptr;
    hipError_t e = hipMalloc(&c->scan_tmp, sizeof(int) * (size_t)(nb + 64));
    if (e != hipSuccess) return e;
    c->scan_tmp_cap = nb;
  }
  hipLaunchKernelGGL(k_block_sums, dim3(nb), dim3(kThreads), 0, c->stream, in, n, c->scan_tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kThreads), 0, c->stream, c->scan_tmp, nb, out + n);
  hipLaunchKernelGGL(k_scan_tiles, dim3(nb), dim3(kThreads), 0, c->stream, in, out, n,
                     c->scan_tmp);
  return hipGetLastError();
}
