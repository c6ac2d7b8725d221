// order.hip - per-domain update order and slot layout.
//
// Inside a domain the contacts are updated sequentially (Sec. 3.1).  The
// order used here is a greedy first-fit colouring of the domain's contacts
// taken in canonical order (two contacts conflict when they share a
// particle; walls never conflict), then (colour, canonical id).  Contacts of
// one colour touch disjoint particles, so updating them at the same time in
// different lanes gives exactly the result of updating them one after the
// other: the colour-major sweep is an exact sequential sweep.
//
// Steps (no limit on the domain size):
//   1. contacts grouped by domain, canonical order kept: stable radix sort of
//      (domain, contact id);
//   2. each domain's particles, ascending: radix sort of (domain, particle)
//      keys of all contact ends, then unique;
//   3. local body indices of every contact (binary search in its domain's
//      particle list);
//   4. one workgroup per domain colours serially (first fit, the order is
//      the definition) with the per-particle colour masks in LDS when the
//      domain fits, and writes the slot arrays: local body indices, contact
//      frame, force-law constants and the initial force records;
//   5. per-particle incidence lists in ascending contact id.
#include <algorithm>

#include "cd_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kBuild = 64;   // one wavefront: the small-domain colouring runs in lockstep
constexpr int kSmall = 512;    // colouring in LDS up to this many contacts and particles

__global__ __launch_bounds__(kThreads) void k_dom_keys(const int* dom, int64_t nc,
                                                      unsigned long long* keys, int* vals) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  keys[c] = (unsigned long long)dom[c];
  vals[c] = (int)c;
}

// First index of each domain d in 0..P in the contacts sorted by domain
// (binary search over the sorted keys): the domain's contact range.
__global__ __launch_bounds__(kThreads) void k_dom_bounds(const unsigned long long* keys,
                                                        int64_t m, int P, int* start) {
  const int d = blockIdx.x * kThreads + threadIdx.x;
  if (d > P) return;
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < (unsigned long long)d) lo = mid + 1;
    else hi = mid;
  }
  start[d] = (int)lo;
}

// Distinct domains of particle p's incident contacts (its domain entries),
// in increasing domain order; returns their count.
__device__ inline int particle_domains(const int* inc_ptr, const int* inc, const int* dom, int p,
                                       int* out, int cap_out) {
  int k = 0;
  for (int e = inc_ptr[p]; e < inc_ptr[p + 1]; ++e) {
    const int d = dom[inc[e] >> 1];
    int q = 0;
    while (q < k && out[q] < d) ++q;
    if (q < k && out[q] == d) continue;
    if (k == cap_out) return -1;
    for (int r = k; r > q; --r) out[r] = out[r - 1];
    out[q] = d;
    ++k;
  }
  return k;
}

// slots k >= count of the pair arrays: a key past every domain
__global__ __launch_bounds__(kThreads) void k_pad_keys(const int* count, int64_t m,
                                                      unsigned long long* keys, int* vals) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= m || k < *count) return;
  keys[k] = ~0ull;
  vals[k] = 0;
}

constexpr int kMaxPartDomains = 32;   // distinct domains of one particle's contacts

__global__ __launch_bounds__(kThreads) void k_pdom_count(const int* inc_ptr, const int* inc,
                                                        const int* dom, int64_t n, int* count,
                                                        DomainStats* stats) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  int ds[kMaxPartDomains];
  int k = particle_domains(inc_ptr, inc, dom, (int)p, ds, kMaxPartDomains);
  if (k < 0) {
    atomicMax(&stats->overflow, 3);
    k = 0;
  }
  count[p] = k;
}

// (domain, particle) pairs in particle-major order; a stable sort by domain
// then gives every domain's particles in increasing id
__global__ __launch_bounds__(kThreads) void k_pdom_write(const int* inc_ptr, const int* inc,
                                                        const int* dom, int64_t n, const int* off,
                                                        unsigned long long* keys, int* vals) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  int ds[kMaxPartDomains];
  const int k = particle_domains(inc_ptr, inc, dom, (int)p, ds, kMaxPartDomains);
  if (k < 0) return;
  const int o = off[p];
  for (int q = 0; q < k; ++q) {
    keys[o + q] = (unsigned long long)ds[q];
    vals[o + q] = (int)p;
  }
}

__device__ inline int lower_bound_i(const int* a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kThreads) void k_local_index(const int* bucket, const int* dom,
                                                         const int* ci, const int* cj,
                                                         int64_t nc, int64_t n, const int* dp,
                                                         const int* dp_start, int* qla,
                                                         int* qlb) {
  int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= nc) return;
  int c = bucket[q];
  int d = dom[c];
  int ps = dp_start[d], np = dp_start[d + 1] - ps;
  // (clamped: only a particle dropped by a reported overflow is missing)
  auto find = [&](int v) {
    const int k = lower_bound_i(dp + ps, np, v);
    return k < np ? k : (np > 0 ? np - 1 : 0);
  };
  qla[q] = find(ci[c]);
  int b = cj[c];
  qlb[q] = b < n ? find(b) : -1 - (int)(b - n);
}

struct BuildArgs {
  const int* dom_start;
  const int* bucket;
  const int* dp_start;
  const int* qla;
  const int* qlb;
  int* qcol;              // scratch, per bucket position
  int* qpos;              // scratch, per bucket position
  unsigned long long* gmask;   // scratch, per domain particle
  const int* ci;
  const int* cj;
  const double* nrm;
  const double* gap;
  const double* R;        // canonical initial forces (dim x nc)
  const double* r;
  const double* inv_m;
  const double* inv_I;
  int64_t n;
  int64_t nc;
  int64_t cap;
  double dt;
  int clamp;
  int* slot_contact;
  int* contact_slot;
  int* color;
  int2* ab;
  double* geo;
  double* rec0;
  double* rec1;           // the other record array (3D: it carries the normals too)
  int* dcol;
  int* dncol;
  int* ddesc;             // per domain: cs, nct, ps, np, ncol, 0, 0, 0
  DomainStats* stats;
  const unsigned char* par;   // contacts updated in parallel (canonical order), or null
  int levels;                 // colours by level: the bucket order is the caller's order
  int mobile;                 // bit w: wall w has finite mass (its contacts conflict)
  double wim[CD_MAX_WALLS];   // 1/M of each wall (0: prescribed motion)
};

// Checks a caller's contact list (cd_solve_contacts) before any kernel
// indexes with it: 0 <= ci < n, ci < cj < n + W, keys (ci, cj) strictly
// increasing; domains in [0, P); the order a permutation of the contacts
// with non-decreasing domains.  Bits of *fault: 1 list, 2 domains, 4 order.
// `seen` (nc ints) must be zero.
__global__ __launch_bounds__(kThreads) void k_check_inputs(const int* ci, const int* cj,
                                                          int64_t nc, int64_t n, int W,
                                                          const int* dom, int P,
                                                          const int* order, int* seen,
                                                          int* fault) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= nc) return;
  int bad = 0;
  const int a = ci[q], b = cj[q];
  if (a < 0 || (int64_t)a >= n || b <= a || (int64_t)b >= n + W) bad |= 1;
  if (q > 0) {
    const int a0 = ci[q - 1], b0 = cj[q - 1];
    if (a0 > a || (a0 == a && b0 >= b)) bad |= 1;
  }
  if (dom) {
    const int d = dom[q];
    if (d < 0 || d >= P) bad |= 2;
  }
  if (order) {
    const int o = order[q];
    if (o < 0 || (int64_t)o >= nc) {
      bad |= 4;
    } else {
      if (atomicAdd(&seen[o], 1) != 0) bad |= 4;
      if (q > 0) {
        const int o0 = order[q - 1];
        if (o0 >= 0 && (int64_t)o0 < nc && dom) {
          const int d0 = dom[o0], d1 = dom[o];
          if (d0 >= 0 && d0 < P && d1 >= 0 && d1 < P && d0 > d1) bad |= 4;
        }
      }
    }
  }
  if (bad) atomicOr(fault, bad);
}

// The caller's order as the bucket, and its sorted domain keys
// contacts of wall body `body` (flag 1) and, after a scan, their slots
__global__ __launch_bounds__(kThreads) void k_wall_flags(const int* cj, int64_t nc, int body,
                                                        int* flag) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c < nc) flag[c] = cj[c] == body ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_wall_scatter(const int* flag, const int* pos,
                                                          int64_t nc, const int* contact_slot,
                                                          int* out, int* count) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c < nc && flag[c]) out[pos[c]] = contact_slot[c];
  if (c == 0) *count = pos[nc];
}

__global__ __launch_bounds__(kThreads) void k_order_keys(const int* order, const int* dom,
                                                        int64_t nc, unsigned long long* keys,
                                                        int* bucket) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= nc) return;
  const int c = order[q];
  bucket[q] = c;
  keys[q] = (unsigned long long)dom[c];
}

// Greedy first-fit colouring of a domain's contacts in canonical order
// (serial by definition; thread 0): col[k], and rank[k] = number of earlier
// contacts of the same colour, so that the stable order by colour is
// pos[k] = offset[col[k]] + rank[k].  Returns the colour count, or -1 when a
// contact finds all CD_MAX_COLORS colours taken.  MASK/LA/LB/COL/RANK are
// LDS arrays in the small path and global scratch in the large one.  In
// the mixed update (Sec. 2.3) a contact with par(k) takes colour 0 and the
// masks start with colour 0 taken, so that the others colour from 1.
// The colour a contact takes given the colours `used` by earlier contacts on
// its bodies: first fit, or (LEVELS, for an update order the caller gives)
// one above the highest, so that every contact follows all earlier contacts
// it shares a body with and each colour holds contacts of disjoint bodies:
// colour by colour, ties by position, is then the same sequential order.
// Returns CD_MAX_COLORS when none is left.
__device__ inline int colour_of(unsigned long long used, bool levels) {
  if (levels) return used == 0ull ? 0 : 64 - __clzll((long long)used);
  return used == ~0ull ? CD_MAX_COLORS : __ffsll((long long)~used) - 1;
}

template <typename M, typename I, typename C, typename Par>
__device__ inline int colour_serial(int nct, M* mask, const I* la_s, const I* lb_s, C* col_s,
                                    C* rank_s, int* cnt, Par&& par, bool levels, int mobile,
                                    unsigned long long wmask0) {
  int ncol = 0;
  // colour sets of the walls of finite mass (bodies whose contacts conflict)
  unsigned long long wmask[CD_MAX_WALLS];
  for (int q = 0; q < CD_MAX_WALLS; ++q) wmask[q] = wmask0;
  for (int k = 0; k < nct; ++k) {
    if (par(k)) {
      col_s[k] = (C)0;
      rank_s[k] = (C)cnt[0];
      cnt[0] += 1;
      if (ncol < 1) ncol = 1;
      continue;
    }
    const int la = la_s[k], lb = lb_s[k];
    const bool bw = lb < 0 && ((mobile >> (-1 - lb)) & 1);
    const unsigned long long used =
        mask[la] | (lb >= 0 ? (unsigned long long)mask[lb] : (bw ? wmask[-1 - lb] : 0ull));
    const int col = colour_of(used, levels);
    if (col >= CD_MAX_COLORS) return -1;
    col_s[k] = (C)col;
    rank_s[k] = (C)cnt[col];
    cnt[col] += 1;
    mask[la] |= 1ull << col;
    if (lb >= 0) mask[lb] |= 1ull << col;
    else if (bw) wmask[-1 - lb] |= 1ull << col;
    if (col + 1 > ncol) ncol = col + 1;
  }
  return ncol;
}

// The same colouring by one whole wavefront in lockstep (small domains,
// LDS arrays): every lane follows the same contact, lane q keeps the count
// of colour q in a register, and each step costs one round trip to LDS
// (the next contact's bodies are read one step ahead).
__device__ inline int colour_wave(int nct, unsigned long long* mask, const int* la_s,
                                  const int* lb_s, short* col_s, short* rank_s, int* cnt_out,
                                  const unsigned char* par, bool levels, int mobile,
                                  unsigned long long* wmask) {
  static_assert(CD_MAX_COLORS == 64, "one lane per colour");
  const int lane = threadIdx.x & 63;
  int cnt = 0;   // contacts of colour `lane` so far
  int ncol = 0;
  int la = nct > 0 ? la_s[0] : 0, lb = nct > 0 ? lb_s[0] : -1;
  for (int k = 0; k < nct; ++k) {
    const int la_n = k + 1 < nct ? la_s[k + 1] : 0;
    const int lb_n = k + 1 < nct ? lb_s[k + 1] : -1;
    if (par && par[k]) {
      // updated in parallel: colour 0, no mask (the same for every lane)
      const int rank = __builtin_amdgcn_readlane(cnt, 0);
      if (lane == 0) {
        ++cnt;
        col_s[k] = 0;
        rank_s[k] = (short)rank;
      }
      if (ncol < 1) ncol = 1;
      la = la_n;
      lb = lb_n;
      continue;
    }
    // a wall of finite mass is a body: its contacts conflict
    const bool bw = lb < 0 && ((mobile >> (-1 - lb)) & 1);
    const unsigned long long ma = mask[la],
                             mb = lb >= 0 ? mask[lb] : (bw ? wmask[-1 - lb] : 0ull);
    const unsigned long long used = ma | mb;
    const int col = __builtin_amdgcn_readfirstlane(colour_of(used, levels));
    if (col >= CD_MAX_COLORS) return -1;
    const int rank = __builtin_amdgcn_readlane(cnt, col);
    if (lane == col) ++cnt;
    if (lane == 0) {
      col_s[k] = (short)col;
      rank_s[k] = (short)rank;
      mask[la] = ma | (1ull << col);
      if (lb >= 0) mask[lb] = mb | (1ull << col);
      else if (bw) wmask[-1 - lb] = mb | (1ull << col);
    }
    if (col + 1 > ncol) ncol = col + 1;
    la = la_n;
    lb = lb_n;
  }
  cnt_out[lane] = cnt;
  return ncol;
}

// Contacts updated in parallel in the mixed update (Sec. 2.3): those whose
// pair number u = top 53 bits of SplitMix64(SplitMix64(SplitMix64(seed) ^ i)
// ^ j) (Steele, Lea and Flood 2014) falls below p.
__device__ inline unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kThreads) void k_par_flags(const int* ci, const int* cj, int64_t nc,
                                                       double p, unsigned long long seed,
                                                       unsigned char* par) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  const unsigned long long h =
      splitmix64(splitmix64(splitmix64(seed) ^ (unsigned long long)(long long)ci[c]) ^
                 (unsigned long long)(long long)cj[c]);
  const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
  par[c] = u < p ? 1 : 0;
}

// Largest colour count, contacts, particle entries and LDS staging over
// all domain descriptors, by one workgroup (a same-address atomic from
// every domain workgroup would serialise).
constexpr int kStats = 1024;
__global__ __launch_bounds__(kStats) void k_dom_stats(const int* ddesc, int P, int stage_doubles,
                                                     DomainStats* stats) {
  __shared__ int sh[4][kStats / 64];
  int mc = 0, mn = 0, mp = 0;
  for (int d = threadIdx.x; d < P; d += kStats) {
    const int* dd = ddesc + 8 * (int64_t)d;
    mn = max(mn, dd[1]);
    mp = max(mp, dd[3]);
    mc = max(mc, dd[4]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mc = max(mc, __shfl_xor(mc, off, 64));
    mn = max(mn, __shfl_xor(mn, off, 64));
    mp = max(mp, __shfl_xor(mp, off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = mc;
    sh[1][w] = mn;
    sh[2][w] = mp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kStats / 64; ++k) {
      mc = max(mc, sh[0][k]);
      mn = max(mn, sh[1][k]);
      mp = max(mp, sh[2][k]);
    }
    stats->max_colors = mc;
    stats->max_contacts = mn;
    stats->max_particles = mp;
    // sweep staging in LDS: per particle V, W, dt/m, dt/I, r
    const long long bytes = 8ll * stage_doubles * mp;
    stats->max_lds = (int)(bytes < 0x7fffffffll ? bytes : 0x7fffffffll);
  }
}

template <int DIM, int SMALL>
__global__ __launch_bounds__(kBuild) void k_dom_build(BuildArgs a) {
  constexpr int REC = cd_rec(DIM);
  __shared__ unsigned long long s_mask[SMALL];
  __shared__ int s_la[SMALL], s_lb[SMALL];
  __shared__ short s_col[SMALL], s_rank[SMALL];
  __shared__ unsigned char s_par[SMALL];
  __shared__ int s_cnt[CD_MAX_COLORS];
  __shared__ int s_coloff[CD_MAX_COLORS + 1];
  __shared__ int s_ncol;
  __shared__ unsigned long long s_wmask[CD_MAX_WALLS];
  __shared__ int s_wtouch;

  const int d = blockIdx.x;
  const int cs = a.dom_start[d], nct = a.dom_start[d + 1] - cs;
  const int ps = a.dp_start[d], np = a.dp_start[d + 1] - ps;
  if (nct > 0 && np == 0) {
    // only after a reported overflow (particles dropped from the entries)
    if (threadIdx.x == 0) atomicMax(&a.stats->overflow, 3);
    return;
  }
  const bool small = nct <= SMALL && np <= SMALL;
  for (int q = threadIdx.x; q < CD_MAX_COLORS; q += blockDim.x) s_cnt[q] = 0;
  // mixed update: colour 0 is reserved for the contacts updated in parallel
  const unsigned long long mask0 = a.par ? 1ull : 0ull;
  for (int q = threadIdx.x; q < CD_MAX_WALLS; q += blockDim.x) s_wmask[q] = mask0;
  if (threadIdx.x == 0) s_wtouch = 0;
  if (small) {
    for (int k = threadIdx.x; k < np; k += blockDim.x) s_mask[k] = mask0;
    for (int k = threadIdx.x; k < nct; k += blockDim.x) {
      s_la[k] = a.qla[cs + k];
      s_lb[k] = a.qlb[cs + k];
      s_par[k] = a.par ? a.par[a.bucket[cs + k]] : 0;
    }
  } else {
    for (int k = threadIdx.x; k < np; k += blockDim.x) a.gmask[ps + k] = mask0;
  }
  __syncthreads();
  int ncol_w = 0;
  if (small) ncol_w = colour_wave(nct, s_mask, s_la, s_lb, s_col, s_rank, s_cnt,
                                  a.par ? s_par : nullptr, a.levels != 0, a.mobile, s_wmask);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned char* par = a.par;
    const int* bk = a.bucket + cs;
    auto is_par = [&](int k) { return par != nullptr && par[bk[k]] != 0; };
    const int ncol = small ? ncol_w
                           : colour_serial(nct, a.gmask + ps, a.qla + cs, a.qlb + cs,
                                           a.qcol + cs, a.qpos + cs, s_cnt, is_par,
                                           a.levels != 0, a.mobile, mask0);
    s_coloff[0] = 0;
    for (int q = 0; q < ncol; ++q) s_coloff[q + 1] = s_coloff[q] + s_cnt[q];
    s_ncol = ncol;
  }
  __syncthreads();
  if (s_ncol < 0) {
    if (threadIdx.x == 0) atomicMax(&a.stats->overflow, 2);
    return;
  }
  // the walls of finite mass this domain touches (its sweep recomputes their
  // velocity in the exchange)
  if (a.mobile) {
    for (int k = threadIdx.x; k < nct; k += blockDim.x) {
      const int lb = small ? s_lb[k] : a.qlb[cs + k];
      if (lb < 0 && ((a.mobile >> (-1 - lb)) & 1)) atomicOr(&s_wtouch, 1 << (-1 - lb));
    }
    __syncthreads();
  }
  // stable order by colour
  int* pos = a.qpos + cs;
  if (small)
    for (int k = threadIdx.x; k < nct; k += blockDim.x) pos[k] = s_coloff[s_col[k]] + s_rank[k];
  else
    for (int k = threadIdx.x; k < nct; k += blockDim.x) pos[k] = s_coloff[a.qcol[cs + k]] + pos[k];
  __syncthreads();
  const int ncol = s_ncol;
  if (threadIdx.x == 0) {
    int* dd = a.ddesc + 8 * (int64_t)d;
    dd[0] = cs;
    dd[1] = nct;
    dd[2] = ps;
    dd[3] = np;
    dd[4] = ncol;
    int widest = 0;   // the largest colour (of the sequential ones in the mixed update)
    for (int q = a.par ? 1 : 0; q < ncol; ++q) widest = max(widest, s_coloff[q + 1] - s_coloff[q]);
    dd[5] = widest;
    dd[6] = s_wtouch;
    dd[7] = 0;
    a.dncol[d] = ncol;
  }
  for (int q = threadIdx.x; q <= CD_MAX_COLORS; q += blockDim.x)
    a.dcol[(int64_t)d * (CD_MAX_COLORS + 1) + q] = q <= ncol ? s_coloff[q] : nct;
  // slot arrays
  const int64_t nc = a.nc, cap = a.cap, nn = a.n;
  for (int k = threadIdx.x; k < nct; k += blockDim.x) {
    const int c = a.bucket[cs + k];
    const int64_t s = cs + pos[k];
    const int i = a.ci[c], j = a.cj[c];
    a.slot_contact[s] = c;
    a.contact_slot[c] = (int)s;
    a.color[c] = small ? s_col[k] : a.qcol[cs + k];
    a.ab[s] = make_int2(a.qla[cs + k], a.qlb[cs + k]);
    double n3[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < DIM; ++q) n3[q] = a.nrm[q * nc + c];
    double t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
    if (DIM == 2) {
      t1[0] = -n3[1];
      t1[1] = n3[0];
    } else {
      // tangent basis of Duff et al., JCGT 6(1), 2017 (t1 x t2 = n)
      double sign = copysign(1.0, n3[2]);
      double aa = -1.0 / (sign + n3[2]);
      double bb = n3[0] * n3[1] * aa;
      t1[0] = 1.0 + sign * n3[0] * n3[0] * aa;
      t1[1] = sign * bb;
      t1[2] = -sign * n3[0];
      t2[0] = bb;
      t2[1] = sign + n3[1] * n3[1] * aa;
      t2[2] = -n3[1];
    }
    // pair inverse mass matrix in the contact frame: M^-1 = w_n nn + w_t (1 - nn)
    double wn = a.inv_m[i] + (j < nn ? a.inv_m[j] : 0.0);
    double wt = wn + (a.r[i] * a.r[i]) * a.inv_I[i];
    wt = wt + (j < nn ? (a.r[j] * a.r[j]) * a.inv_I[j] : 0.0);
    if (j >= nn && ((a.mobile >> (j - nn)) & 1)) {
      // a wall of finite mass moves along its normal only: 1/M adds to the
      // normal term, nothing to the tangential one
      wn = a.inv_m[i] + a.wim[j - nn];
      wt = a.inv_m[i] + (a.r[i] * a.r[i]) * a.inv_I[i];
    }
    double ge = a.gap[c];
    if (a.clamp && ge < 0.0) ge = 0.0;
    double* g = a.geo;
    for (int q = 0; q < DIM; ++q) g[(G_N0 + q) * cap + s] = n3[q];
    if (DIM == 3) {
      for (int q = 0; q < 3; ++q) {
        g[(G_T10 + q) * cap + s] = t1[q];
        g[(G_T20 + q) * cap + s] = t2[q];
      }
    }
    double dwn = a.dt * wn, dwt = a.dt * wt;
    g[G_GDT * cap + s] = ge / a.dt;
    g[G_DWN * cap + s] = dwn;
    g[G_DWT * cap + s] = dwt;
    g[G_KN * cap + s] = 1.0 / dwn;
    g[G_KT * cap + s] = 1.0 / dwt;
    // initial force record
    double* rc = a.rec0 + s * REC;
    double rn = a.R[c], r1 = a.R[nc + c], r2 = DIM == 3 ? a.R[2 * nc + c] : 0.0;
    if (DIM == 2) {
      rc[0] = rn;
      rc[1] = r1;
      rc[2] = rn * n3[0] + r1 * t1[0];
      rc[3] = rn * n3[1] + r1 * t1[1];
    } else {
      // the frame force; F and n x R are rebuilt from it and the normal
      rc[0] = rn;
      rc[1] = r1;
      rc[2] = r2;
      rc[3] = 0.0;
      // the normal half, in both record arrays
      double* n4 = rc + 4;
      double* m4 = a.rec1 + s * REC + 4;
      for (int q = 0; q < 3; ++q) n4[q] = m4[q] = n3[q];
      n4[3] = m4[3] = 0.0;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_inc_count(const int* ci, const int* cj, int64_t nc,
                                                       int64_t n, int* count) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  atomicAdd(&count[ci[c]], 1);
  if (cj[c] < n) atomicAdd(&count[cj[c]], 1);
}

__global__ __launch_bounds__(kThreads) void k_inc_fill(const int* ci, const int* cj, int64_t nc,
                                                      int64_t n, const int* ptr, int* cursor,
                                                      int* inc) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  int a = ci[c];
  inc[ptr[a] + atomicAdd(&cursor[a], 1)] = (int)(2 * c);
  int b = cj[c];
  if (b < n) inc[ptr[b] + atomicAdd(&cursor[b], 1)] = (int)(2 * c + 1);
}

// sort each particle's incidences by contact id
__global__ __launch_bounds__(kThreads) void k_inc_sort(int64_t n, const int* ptr, int* inc) {
  int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  int s0 = ptr[p], s1 = ptr[p + 1];
  for (int k = s0 + 1; k < s1; ++k) {
    int v = inc[k];
    int q = k;
    while (q > s0 && inc[q - 1] > v) {
      inc[q] = inc[q - 1];
      --q;
    }
    inc[q] = v;
  }
}

// the incidences refer to slots instead of contacts (order kept)
__global__ __launch_bounds__(kThreads) void k_inc_slots(const int* total, int64_t m,
                                                       const int* contact_slot, int* inc) {
  int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= m || k >= *total) return;
  const int v = inc[k];
  inc[k] = 2 * contact_slot[v >> 1] + (v & 1);
}

// domain particle entries in domain order: base data (SoA, stride E) and
// the incidence count of the particle
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_dp_entries(const int* dp, const int* dp_start, int P,
                                                        int64_t E, const double* v,
                                                        const double* w, const double* f,
                                                        const double* t, const double* dtim,
                                                        const double* dtii, const double* r,
                                                        const int* inc_ptr, int64_t n,
                                                        double* dpb, int* count,
                                                        DomainStats* stats) {
  constexpr int DR = DIM == 2 ? 1 : 3;
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E) return;
  const int total = dp_start[P];
  if (e == 0) stats->dp_total = total;
  if (e >= total) {
    count[e] = 0;
    return;
  }
  const int p = dp[e];
  int q = 0;
  for (int k = 0; k < DIM; ++k) dpb[(q++) * E + e] = v[k * n + p];
  for (int k = 0; k < DR; ++k) dpb[(q++) * E + e] = w[k * n + p];
  for (int k = 0; k < DIM; ++k) dpb[(q++) * E + e] = f[k * n + p];
  for (int k = 0; k < DR; ++k) dpb[(q++) * E + e] = t[k * n + p];
  dpb[(q++) * E + e] = dtim[p];
  dpb[(q++) * E + e] = dtii[p];
  dpb[(q++) * E + e] = r[p];
  count[e] = inc_ptr[p + 1] - inc_ptr[p];
}

__global__ void k_dinc_total(const int* dinc_ptr, int64_t E, DomainStats* stats) {
  stats->dinc_total = dinc_ptr[E];
}

__global__ __launch_bounds__(kThreads) void k_dinc_fill(const int* dp, const int* dp_start, int P,
                                                       int64_t E, const int* inc_ptr,
                                                       const int* inc, const int* dinc_ptr,
                                                       int* dinc) {
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E || e >= dp_start[P]) return;
  const int p = dp[e];
  const int s0 = inc_ptr[p], s1 = inc_ptr[p + 1];
  int o = dinc_ptr[e];
  for (int k = s0; k < s1; ++k) dinc[o++] = inc[k];
}

// fixed-width incidence rows: the first KW incident slots of each domain
// particle entry, padded with -1; a row starting with -2 marks an entry with
// more than KW incidences, whose list is read through dinc_ptr / dinc
__global__ __launch_bounds__(kThreads) void k_dinc_rows(const int* dp, const int* dp_start, int P,
                                                       int64_t E, int KW, const int* inc_ptr,
                                                       const int* inc, int* rows) {
  // rows are stored as KW/4 planes of int4, plane q holding entries 4q..4q+3
  // of every particle entry: rows[(q E + e) 4 + k]
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E || e >= dp_start[P]) return;
  const int p = dp[e];
  const int s0 = inc_ptr[p], deg = inc_ptr[p + 1] - s0;
  for (int q = 0; q < KW / 4; ++q) {
    int v[4];
    for (int k = 0; k < 4; ++k) {
      const int x = 4 * q + k;
      v[k] = deg > KW ? (x == 0 ? -2 : -1) : (x < deg ? inc[s0 + x] : -1);
    }
    *(int4*)(rows + (q * E + e) * 4) = make_int4(v[0], v[1], v[2], v[3]);
  }
}

// The domain of particle entry e < dp_start[P]: the d with
// dp_start[d] <= e < dp_start[d + 1] (an empty domain has no entry).
__device__ inline int entry_domain(const int* dp_start, int P, int e) {
  int lo = 0, hi = P;
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (dp_start[m] <= e) lo = m;
    else hi = m;
  }
  return lo;
}

// Foreign incidences of each domain particle entry: the incident slots that
// belong to another domain (their forces come from the exchange).  The
// incidence lists hold slots at this point.
__global__ __launch_bounds__(kThreads) void k_halo_count(const int* dp, const int* dp_start, int P,
                                                        int64_t E, const int* dom_start,
                                                        const int* inc_ptr, const int* inc,
                                                        int* count) {
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E) return;
  if (e >= dp_start[P]) {
    count[e] = 0;
    return;
  }
  const int d = entry_domain(dp_start, P, (int)e);
  const int cs = dom_start[d], ce = dom_start[d + 1];
  const int p = dp[e];
  int m = 0;
  for (int x = inc_ptr[p]; x < inc_ptr[p + 1]; ++x) {
    const int s = inc[x] >> 1;
    m += (s < cs || s >= ce) ? 1 : 0;
  }
  count[e] = m;
}

// Per domain: the range of its foreign incidences in the list, and the
// largest count and staged sweep size over all domains (one workgroup, as
// k_dom_stats).  ps, sw, hw: doubles staged per particle entry, slot (without
// a per-slot friction coefficient, which may be set later) and foreign
// incidence.
__global__ __launch_bounds__(kStats) void k_halo_dom(const int* dp_start, const int* ddesc, int P,
                                                    const int* hoff, int ps, int sw, int hw,
                                                    int2* dhalo, DomainStats* stats) {
  __shared__ long long sh[4][kStats / 64];
  long long mh = 0, mb = 0, m0 = 0, mu = 0;
  for (int d = threadIdx.x; d < P; d += kStats) {
    const int hs = hoff[dp_start[d]];
    const int nh = hoff[dp_start[d + 1]] - hs;
    dhalo[d] = make_int2(hs, nh);
    const int* dd = ddesc + 8 * (int64_t)d;
    const long long b0 = 8ll * ((long long)ps * dd[3] + (long long)sw * dd[1]);
    mh = max(mh, (long long)nh);
    mb = max(mb, b0 + 8ll * hw * nh);
    m0 = max(m0, b0);
    // shared layout: particle records and foreign forces in one area
    const long long pa = (long long)ps * dd[3], ha = (long long)hw * nh;
    const long long bu = 8ll * ((long long)sw * dd[1] + (pa > ha ? pa : ha));
    mu = max(mu, dd[3] <= kUnionMax ? bu : b0 + 8ll * hw * nh);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mh = max(mh, __shfl_xor(mh, off, 64));
    mb = max(mb, __shfl_xor(mb, off, 64));
    m0 = max(m0, __shfl_xor(m0, off, 64));
    mu = max(mu, __shfl_xor(mu, off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = mh;
    sh[1][w] = mb;
    sh[2][w] = m0;
    sh[3][w] = mu;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kStats / 64; ++k) {
      mh = max(mh, sh[0][k]);
      mb = max(mb, sh[1][k]);
      m0 = max(m0, sh[2][k]);
      mu = max(mu, sh[3][k]);
    }
    stats->max_halo = (int)mh;
    stats->max_stage = (int)(mb < 0x7fffffffll ? mb : 0x7fffffffll);
    stats->max_stage0 = (int)(m0 < 0x7fffffffll ? m0 : 0x7fffffffll);
    stats->max_stage_u = (int)(mu < 0x7fffffffll ? mu : 0x7fffffffll);
  }
}

// The foreign incidences' slots, entry by entry in incidence (row) order
__global__ __launch_bounds__(kThreads) void k_halo_fill(const int* dp, const int* dp_start, int P,
                                                       int64_t E, const int* dom_start,
                                                       const int* inc_ptr, const int* inc,
                                                       const int* hoff, const int2* dhalo,
                                                       int hstride, int* halo, int* hpad) {
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E || e >= dp_start[P]) return;
  const int d = entry_domain(dp_start, P, (int)e);
  const int cs = dom_start[d], ce = dom_start[d + 1];
  const int p = dp[e];
  const int hs = dhalo[d].x;
  int o = hoff[e];
  for (int x = inc_ptr[p]; x < inc_ptr[p + 1]; ++x) {
    const int s = inc[x] >> 1;
    if (s < cs || s >= ce) {
      // list index o is the domain's foreign incidence o - hs
      if (o - hs < hstride) hpad[(int64_t)d * hstride + (o - hs)] = s;
      halo[o++] = s;
    }
  }
}

int bits_for(unsigned long long maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0ull) ++b;
  return ((b + 7) / 8) * 8;
}

}  // namespace

hipError_t cd_launch_order(cd_ctx* c) {
  const int64_t nc = c->nc;
  const int64_t n = c->n;
  const int P = c->P;
  hipError_t e;
  e = hipMemsetAsync(c->d_stats, 0, offsetof(DomainStats, scan_fault), c->stream);
  if (e != hipSuccess) return e;
  // 1. contacts by domain, canonical order kept (stable sort); each
  //    domain's contact range from the sorted keys
  unsigned long long* ko = c->sort_keys[0];
  int* vo = c->sort_vals[0];
  if (nc > 0 && c->given_order) {
    // a caller's order (checked): its domain segments are already sorted
    hipLaunchKernelGGL(k_order_keys, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0,
                       c->stream, c->given_order, c->dom, nc, c->sort_keys[0], c->bucket);
  } else if (nc > 0) {
    // the contact ids are sorted in place in `bucket` (an even number of
    // passes ends there; otherwise the result is copied back)
    hipLaunchKernelGGL(k_dom_keys, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->dom, nc, c->sort_keys[0], c->bucket);
    e = cd_radix_sort(c, c->sort_keys[0], c->bucket, c->sort_keys[1], c->sort_vals[1], nc,
                      bits_for((unsigned long long)(P - 1)), &ko, &vo);
    if (e != hipSuccess) return e;
    if (vo != c->bucket) {
      e = hipMemcpyAsync(c->bucket, vo, sizeof(int) * (size_t)nc, hipMemcpyDeviceToDevice,
                         c->stream);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_dom_bounds, dim3(cd_blocks(P + 1, kThreads)), dim3(kThreads), 0, c->stream,
                     ko, nc, P, c->dom_start);
  // 2. incidence lists: each particle's contacts in increasing id
  e = hipMemsetAsync(c->inc_count, 0, sizeof(int) * (size_t)(n + 1), c->stream);
  if (e != hipSuccess) return e;
  if (nc > 0)
    hipLaunchKernelGGL(k_inc_count, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->ci, c->cj, nc, n, c->inc_count);
  e = cd_scan_exclusive(c, c->inc_count, c->inc_ptr, n);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(c->inc_cursor, 0, sizeof(int) * (size_t)(n + 1), c->stream);
  if (e != hipSuccess) return e;
  if (nc > 0)
    hipLaunchKernelGGL(k_inc_fill, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->ci, c->cj, nc, n, c->inc_ptr, c->inc_cursor, c->inc);
  hipLaunchKernelGGL(k_inc_sort, dim3(cd_blocks(n, kThreads)), dim3(kThreads), 0, c->stream, n,
                     c->inc_ptr, c->inc);
  // 3. each domain's particles: per particle the distinct domains of its
  //    contacts as (domain, particle) pairs in particle order, sorted stably
  //    by domain (the per-particle counts and offsets reuse the incidence
  //    cursor and count arrays, free by now)
  int* pcount = c->inc_cursor;
  int* poff = c->inc_count;
  hipLaunchKernelGGL(k_pdom_count, dim3(cd_blocks(n, kThreads)), dim3(kThreads), 0, c->stream,
                     c->inc_ptr, c->inc, c->dom, n, pcount, c->d_stats);
  e = cd_scan_exclusive(c, pcount, poff, n);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pdom_write, dim3(cd_blocks(n, kThreads)), dim3(kThreads), 0, c->stream,
                     c->inc_ptr, c->inc, c->dom, n, poff, c->sort_keys[0], c->dp);
  // the number of pairs is poff[n] (at most 2 n_c), known on the device only:
  // the sort covers the 2 n_c slots, the unused tail keyed past every domain
  {
    const int64_t m = 2 * nc;
    if (m > 0) {
      // sorted in place in `dp` when the pass count is even
      hipLaunchKernelGGL(k_pad_keys, dim3(cd_blocks(m, kThreads)), dim3(kThreads), 0, c->stream,
                         poff + n, m, c->sort_keys[0], c->dp);
      e = cd_radix_sort(c, c->sort_keys[0], c->dp, c->sort_keys[1], c->sort_vals[1], m,
                        bits_for((unsigned long long)P), &ko, &vo);
      if (e != hipSuccess) return e;
      if (vo != c->dp) {
        e = hipMemcpyAsync(c->dp, vo, sizeof(int) * (size_t)m, hipMemcpyDeviceToDevice,
                           c->stream);
        if (e != hipSuccess) return e;
      }
    }
    hipLaunchKernelGGL(k_dom_bounds, dim3(cd_blocks(P + 1, kThreads)), dim3(kThreads), 0,
                       c->stream, ko, m, P, c->dp_start);
  }
  // 3. local body indices
  if (nc > 0)
    hipLaunchKernelGGL(k_local_index, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->bucket, c->dom, c->ci, c->cj, nc, n, c->dp, c->dp_start, c->q_la,
                       c->q_lb);
  // 4. colouring and slots
  // mixed update (Sec. 2.3): the contacts updated in parallel
  const unsigned char* par = nullptr;
  if (c->mixed_p >= 0.0) {
    if (c->par_cap < nc || !c->par) {
      if (c->par) (void)hipFree(c->par);
      c->par = nullptr;
      c->par_cap = 0;
      e = hipMalloc((void**)&c->par, (size_t)(c->cap > nc ? c->cap : nc) + 1);
      if (e != hipSuccess) return e;
      c->par_cap = c->cap > nc ? c->cap : nc;
    }
    if (nc > 0)
      hipLaunchKernelGGL(k_par_flags, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0,
                         c->stream, c->ci, c->cj, nc, c->mixed_p, c->mixed_seed, c->par);
    par = c->par;
  }
  c->order_mixed = par != nullptr;
  BuildArgs a;
  a.par = par;
  a.levels = c->given_order != nullptr;
  a.mobile = c->mobile_mask;
  for (int q = 0; q < CD_MAX_WALLS; ++q) a.wim[q] = c->wim[q];
  a.dom_start = c->dom_start;
  a.bucket = c->bucket;
  a.dp_start = c->dp_start;
  a.qla = c->q_la;
  a.qlb = c->q_lb;
  a.qcol = c->q_col;
  a.qpos = c->q_pos;
  a.gmask = c->g_mask;
  a.ci = c->ci;
  a.cj = c->cj;
  a.nrm = c->nrm;
  a.gap = c->gap;
  a.R = c->R;
  a.r = c->r;
  a.inv_m = c->inv_m;
  a.inv_I = c->inv_I;
  a.n = n;
  a.nc = nc;
  a.cap = c->cap;
  a.dt = c->p.dt;
  a.clamp = c->p.overlap_mode == 0;
  a.slot_contact = c->slot_contact;
  a.contact_slot = c->contact_slot;
  a.color = c->color;
  a.ab = c->slot_ab;
  a.geo = c->geo;
  a.rec0 = c->rec[0];
  a.rec1 = c->rec[1];
  a.dcol = c->dcol;
  a.dncol = c->dncol;
  a.ddesc = c->ddesc;
  a.stats = c->d_stats;
  // domains that fit colour in LDS; when they average at most 96 contacts
  // and particles the LDS arrays hold 128 of each (2.8 KB instead of 11 KB,
  // so that some 30 workgroups share a CU instead of 14), a larger domain
  // then takes the global-memory colouring, which gives the same colours
  const bool few = nc <= (int64_t)96 * P && n <= (int64_t)96 * P;
  if (c->dim == 2) {
    if (few) hipLaunchKernelGGL((k_dom_build<2, 128>), dim3(P), dim3(kBuild), 0, c->stream, a);
    else hipLaunchKernelGGL((k_dom_build<2, kSmall>), dim3(P), dim3(kBuild), 0, c->stream, a);
  } else {
    if (few) hipLaunchKernelGGL((k_dom_build<3, 128>), dim3(P), dim3(kBuild), 0, c->stream, a);
    else hipLaunchKernelGGL((k_dom_build<3, kSmall>), dim3(P), dim3(kBuild), 0, c->stream, a);
  }
  hipLaunchKernelGGL(k_dom_stats, dim3(1), dim3(kStats), 0, c->stream, c->ddesc, P,
                     cd_stage_particle(c->dim), c->d_stats);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // 5. the incidence lists refer to slots from here on
  if (nc > 0)
    hipLaunchKernelGGL(k_inc_slots, dim3(cd_blocks(2 * nc, kThreads)), dim3(kThreads), 0,
                       c->stream, c->inc_ptr + n, 2 * nc, c->contact_slot, c->inc);
  // 5b. walls of finite mass: each one's contact slots in ascending contact id
  if (c->mobile_mask) {
    e = cd_launch_wall_lists(c);
    if (e != hipSuccess) return e;
  }
  // 6. domain particle entries and their incidence counts
  const int64_t E = 2 * c->cap;
  if (c->dim == 2)
    hipLaunchKernelGGL(k_dp_entries<2>, dim3(cd_blocks(E, kThreads)), dim3(kThreads), 0, c->stream,
                       c->dp, c->dp_start, P, E, c->v, c->w, c->f, c->t, c->dtim, c->dtii, c->r,
                       c->inc_ptr, n, c->dpb, c->flag, c->d_stats);
  else
    hipLaunchKernelGGL(k_dp_entries<3>, dim3(cd_blocks(E, kThreads)), dim3(kThreads), 0, c->stream,
                       c->dp, c->dp_start, P, E, c->v, c->w, c->f, c->t, c->dtim, c->dtii, c->r,
                       c->inc_ptr, n, c->dpb, c->flag, c->d_stats);
  e = cd_scan_exclusive(c, c->flag, c->dinc_ptr, E);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dinc_total, dim3(1), dim3(1), 0, c->stream, c->dinc_ptr, E, c->d_stats);
  // 7. foreign incidences per entry and domain (their list follows once the
  //    host has sized it)
  hipLaunchKernelGGL(k_halo_count, dim3(cd_blocks(E, kThreads)), dim3(kThreads), 0, c->stream,
                     c->dp, c->dp_start, P, E, c->dom_start, c->inc_ptr, c->inc, c->flag);
  e = cd_scan_exclusive(c, c->flag, c->hoff, E);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_halo_dom, dim3(1), dim3(kStats), 0, c->stream, c->dp_start, c->ddesc, P,
                     c->hoff, cd_stage_particle(c->dim), cd_stage_slot(c->dim, false),
                     cd_stage_halo(c->dim), c->dhalo, c->d_stats);
  return hipGetLastError();
}

hipError_t cd_launch_wall_lists(cd_ctx* c) {
  const int64_t nc = c->nc;
  hipError_t e;
  const int64_t need = (int64_t)c->W * c->cap;
  if (c->wall_slot_cap < need || !c->wall_slot) {
    if (c->wall_slot) (void)hipFree(c->wall_slot);
    c->wall_slot = nullptr;
    c->wall_slot_cap = 0;
    e = hipMalloc((void**)&c->wall_slot, sizeof(int) * (size_t)std::max<int64_t>(need, 1));
    if (e != hipSuccess) return e;
    c->wall_slot_cap = need;
  }
  for (int w = 0; w < c->W; ++w) {
    if (!((c->mobile_mask >> w) & 1)) continue;
    if (nc == 0) {
      e = hipMemsetAsync(c->wall_cnt + w, 0, sizeof(int), c->stream);
      if (e != hipSuccess) return e;
      continue;
    }
    hipLaunchKernelGGL(k_wall_flags, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->cj, nc, (int)(c->n + w), c->flag);
    e = cd_scan_exclusive(c, c->flag, c->flag_scan, nc);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wall_scatter, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0,
                       c->stream, c->flag, c->flag_scan, nc, c->contact_slot,
                       c->wall_slot + (int64_t)w * c->cap, c->wall_cnt + w);
  }
  return hipGetLastError();
}

hipError_t cd_launch_check_inputs(cd_ctx* c, const int* dom, const int* order, int* fault) {
  const int64_t nc = c->nc;
  if (nc <= 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(fault, 0, sizeof(int), c->stream);
  if (e != hipSuccess) return e;
  if (order) {
    e = hipMemsetAsync(c->flag, 0, sizeof(int) * (size_t)nc, c->stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_check_inputs, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                     c->ci, c->cj, nc, c->n, c->W, dom, c->P, order, c->flag, fault);
  return hipGetLastError();
}

hipError_t cd_launch_order_entries(cd_ctx* c) {
  const int64_t E = 2 * c->cap;
  hipLaunchKernelGGL(k_dinc_fill, dim3(cd_blocks(E, kThreads)), dim3(kThreads), 0, c->stream,
                     c->dp, c->dp_start, c->P, E, c->inc_ptr, c->inc, c->dinc_ptr, c->dinc);
  hipLaunchKernelGGL(k_dinc_rows, dim3(cd_blocks(E, kThreads)), dim3(kThreads), 0, c->stream,
                     c->dp, c->dp_start, c->P, E, cd_row_width(c->dim), c->inc_ptr, c->inc,
                     c->drow);
  hipLaunchKernelGGL(k_halo_fill, dim3(cd_blocks(E, kThreads)), dim3(kThreads), 0, c->stream,
                     c->dp, c->dp_start, c->P, E, c->dom_start, c->inc_ptr, c->inc, c->hoff,
                     c->dhalo, c->hstride, c->halo, c->hpad);
  return hipGetLastError();
}
