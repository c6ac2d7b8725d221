// sort.hip - stable least-significant-digit radix sort of (uint64 key,
// int32 value) pairs, 8 bits per pass.  Each pass: per-tile digit
// histograms (digit-major), one exclusive scan over all of them, then a
// stable scatter in which every wavefront ranks equal digits with ballots.
#include "cd_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;

__global__ __launch_bounds__(kThreads) void k_hist(const unsigned long long* keys, int64_t n,
                                                  int shift, int* hist, int nb) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kTile;
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void k_scatter(const unsigned long long* keys_in,
                                                     const int* vals_in,
                                                     unsigned long long* keys_out,
                                                     int* vals_out, int64_t n, int shift,
                                                     const int* offsets, int nb) {
  __shared__ int digit_off[256];
  __shared__ int wave_cnt[kWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  digit_off[threadIdx.x] = offsets[(int64_t)threadIdx.x * nb + blockIdx.x];
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kTile;
  for (int k = 0; k < kItems; ++k) {
    for (int q = threadIdx.x; q < kWaves * 256; q += kThreads) (&wave_cnt[0][0])[q] = 0;
    __syncthreads();
    int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    bool valid = i < n;
    unsigned long long key = valid ? keys_in[i] : 0ull;
    int val = valid ? vals_in[i] : 0;
    int d = (int)((key >> shift) & 255ull);
    // lanes of this wave holding the same digit
    unsigned long long peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      unsigned long long bal = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bal : ~bal;
    }
    int rank = __popcll(peers & lt);
    if (valid && rank == 0) wave_cnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int before = 0;
      for (int w2 = 0; w2 < wave; ++w2) before += wave_cnt[w2][d];
      int pos = digit_off[d] + before + rank;
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    // advance the per-digit offsets by this sub-tile's counts
    {
      int tot = 0;
      for (int w2 = 0; w2 < kWaves; ++w2) tot += wave_cnt[w2][threadIdx.x];
      digit_off[threadIdx.x] += tot;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t cd_radix_sort(cd_ctx* c, unsigned long long* keys, int* vals,
                         unsigned long long* keys_tmp, int* vals_tmp, int64_t n, int bits,
                         unsigned long long** keys_out, int** vals_out) {
  unsigned long long* kin = keys;
  unsigned long long* kout = keys_tmp;
  int* vin = vals;
  int* vout = vals_tmp;
  if (n > 0) {
    int nb = (int)((n + kTile - 1) / kTile);
    int64_t hn = (int64_t)256 * nb;
    if (c->sort_hist_cap < 2 * hn + 1) {
      if (c->sort_hist) (void)hipFree(c->sort_hist);
      c->sort_hist = nullptr;
      hipError_t e = hipMalloc(&c->sort_hist, sizeof(int) * (size_t)(2 * hn + 1));
      if (e != hipSuccess) return e;
      c->sort_hist_cap = 2 * hn + 1;
    }
    int* hist = (int*)c->sort_hist;
    int* off = hist + hn;
    for (int shift = 0; shift < bits; shift += 8) {
      hipLaunchKernelGGL(k_hist, dim3(nb), dim3(kThreads), 0, c->stream, kin, n, shift, hist, nb);
      hipError_t e = cd_scan_exclusive(c, hist, off, hn);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kThreads), 0, c->stream, kin, vin, kout, vout,
                         n, shift, off, nb);
      unsigned long long* tk = kin;
      kin = kout;
      kout = tk;
      int* tv = vin;
      vin = vout;
      vout = tv;
    }
  }
  *keys_out = kin;
  *vals_out = vin;
  return hipGetLastError();
}
