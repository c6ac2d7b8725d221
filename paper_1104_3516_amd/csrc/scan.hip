// scan.hip - exclusive prefix sum of nonnegative int32 counts (out has n+1
// entries, out[n] = total), in one launch: the single-pass scan with
// decoupled look-back of Merrill and Garland (NVIDIA technical report
// NVR-2016-002), written here for 64-wide wavefronts.
//
// Tiles of kTile counts are scanned in the order of a ticket taken from a
// device counter (not blockIdx), so every tile that a tile waits on has
// already started.  Each tile publishes its total at once ("aggregate"),
// then its inclusive prefix once known; a tile finds its exclusive prefix
// by walking back over its predecessors 64 at a time with one wavefront,
// summing aggregates until it meets a published prefix (decoupled
// look-back).  A status word is {epoch:32, prefix flag:1, value:31}; the
// host advances the epoch with every scan, so words left by earlier scans
// read as not yet published and the status array is never cleared between
// scans.  The workgroup holding the launch's last ticket resets the counter
// for the next scan on the stream.
#include "cd_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 32;
constexpr int kTile = kThreads * kItems;
constexpr unsigned long long kPrefixBit = 1ull << 31;
constexpr unsigned long long kValueMask = kPrefixBit - 1;
// polls of one look-back window before giving up (the wait always ends in
// practice: a predecessor only waits on its own predecessors)
constexpr long long kPollLimit = 1ll << 20;

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

__device__ inline unsigned long long status_load(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void status_store(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of tile t (t >= 1) over tiles 0..t-1, by wavefront 0.
__device__ int look_back(const unsigned long long* status, int t, unsigned epoch, int* fault) {
  const int lane = threadIdx.x & 63;
  const unsigned long long tag = (unsigned long long)epoch << 32;
  int excl = 0;
  long long polls = 0;
  for (int base = t - 1;;) {
    // lane L looks at tile base - L; tiles before tile 0 read as a zero
    // prefix (tile 0 always publishes its prefix, so they are never summed)
    const int q = base - lane;
    const unsigned long long w = q >= 0 ? status_load(status + q) : (tag | kPrefixBit);
    const bool valid = (unsigned)(w >> 32) == epoch;
    const unsigned long long pref = __ballot(valid && (w & kPrefixBit));
    const unsigned long long bad = __ballot(!valid);
    // the nearest published prefix ends the walk; every tile up to it
    // must have published at least its aggregate
    const int last = pref ? __builtin_ctzll(pref) : 63;
    const unsigned long long need = last == 63 ? ~0ull : ((2ull << last) - 1);
    if (bad & need) {
      if (++polls <= kPollLimit) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      // give up: flag the fault and finish with what is known, so that
      // every tile still reaches the end of the kernel
      if (lane == 0) __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    polls = 0;
    int v = lane <= last ? (int)(w & kValueMask) : 0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    excl += v;
    if (pref) break;
    base -= 64;
  }
  return excl;
}

__global__ __launch_bounds__(kThreads) void k_scan(const int* in, int* out, int64_t n, int nb,
                                                  unsigned long long* ticket,
                                                  unsigned long long* status, unsigned epoch,
                                                  int* fault) {
  __shared__ int sh[kThreads / 64 + 1];
  __shared__ int s_tile, s_excl;
  if (threadIdx.x == 0) {
    const int t = (int)__hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    // every other tile of this launch already holds its ticket
    if (t == nb - 1) __hip_atomic_store(ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_tile = t;
  }
  __syncthreads();
  const int t = s_tile;
  const int64_t base = (int64_t)t * kTile + (int64_t)threadIdx.x * kItems;
  // a thread's items are consecutive: 16-byte loads where they lie
  // wholly inside the input and it is 16-byte aligned (a tile's first
  // item is, whenever the input is), else one by one
  const bool vec = ((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 15) == 0 &&
                   base + kItems <= n;
  int vals[kItems];
  int s = 0;
  if (vec) {
    static_assert(kItems % 4 == 0, "whole int4 per thread");
    for (int q = 0; q < kItems / 4; ++q) {
      const int4 a = *(const int4*)(in + base + 4 * q);
      vals[4 * q] = a.x;
      vals[4 * q + 1] = a.y;
      vals[4 * q + 2] = a.z;
      vals[4 * q + 3] = a.w;
    }
    for (int k = 0; k < kItems; ++k) s += vals[k];
  } else {
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = base + k;
      vals[k] = i < n ? in[i] : 0;
      s += vals[k];
    }
  }
  int total;
  const int inc = block_inclusive_scan(s, sh, &total);
  if (threadIdx.x < 64) {
    const unsigned long long tag = (unsigned long long)epoch << 32;
    int excl = 0;
    if (t == 0) {
      if (threadIdx.x == 0) status_store(status, tag | kPrefixBit | (unsigned)total);
    } else {
      if (threadIdx.x == 0) status_store(status + t, tag | (unsigned)total);
      excl = look_back(status, t, epoch, fault);
      if (threadIdx.x == 0) status_store(status + t, tag | kPrefixBit | (unsigned)(excl + total));
    }
    if (threadIdx.x == 0) s_excl = excl;
  }
  __syncthreads();
  const int excl = s_excl;
  int run = excl + inc - s;
  if (vec) {
    int o[kItems];
    for (int k = 0; k < kItems; ++k) {
      o[k] = run;
      run += vals[k];
    }
    for (int q = 0; q < kItems / 4; ++q)
      *(int4*)(out + base + 4 * q) = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
  } else {
    for (int k = 0; k < kItems; ++k) {
      const int64_t i = base + k;
      if (i < n) out[i] = run;
      run += vals[k];
    }
  }
  if (t == nb - 1 && threadIdx.x == 0) out[n] = excl + total;
}

}  // namespace

hipError_t cd_scan_exclusive(cd_ctx* c, const int* in, int* out, int64_t n) {
  int nb = (int)((n + kTile - 1) / kTile);
  if (nb < 1) nb = 1;
  hipError_t e;
  if (c->scan_tmp_cap < nb) {
    if (c->scan_tmp) (void)hipFree(c->scan_tmp);
    c->scan_tmp = nullptr;
    c->scan_tmp_cap = 0;
    const int64_t cap = nb + nb / 4 + 64;
    // word 0: ticket counter; status words from word 32 on
    e = hipMalloc(&c->scan_tmp, sizeof(unsigned long long) * (size_t)(cap + 32));
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(c->scan_tmp, 0, sizeof(unsigned long long) * (size_t)(cap + 32), c->stream);
    if (e != hipSuccess) return e;
    c->scan_tmp_cap = cap;
  }
  unsigned epoch = (unsigned)++c->scan_epoch;
  if (epoch == 0) {
    // after 2^32 scans: clear the words so no stale one carries the epoch
    e = hipMemsetAsync(c->scan_tmp + 32, 0, sizeof(unsigned long long) * (size_t)c->scan_tmp_cap,
                       c->stream);
    if (e != hipSuccess) return e;
    epoch = (unsigned)++c->scan_epoch;
  }
  hipLaunchKernelGGL(k_scan, dim3(nb), dim3(kThreads), 0, c->stream, in, out, n, nb, c->scan_tmp,
                     c->scan_tmp + 32, epoch, &c->d_stats->scan_fault);
  return hipGetLastError();
}
