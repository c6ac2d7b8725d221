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
// One workgroup per domain sorts its contacts, builds its particle list
// (ascending id), colours, and writes the slot arrays: local body indices,
// the contact frame and force-law constants, and the initial force records.
// The particle incidence lists (ascending contact id) are built beside it.
#include "cd_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kBuild = 256;

__global__ __launch_bounds__(kThreads) void k_dom_count(const int* dom, int64_t nc, int* count) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c < nc) atomicAdd(&count[dom[c]], 1);
}

__global__ __launch_bounds__(kThreads) void k_dom_scatter(const int* dom, int64_t nc,
                                                         const int* start, int* cursor,
                                                         int* bucket) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  int d = dom[c];
  int pos = atomicAdd(&cursor[d], 1);
  bucket[start[d] + pos] = (int)c;
}

// in-place ascending bitonic sort of n_pow2 ints in shared memory
__device__ void bitonic_sort(int* a, int n_pow2) {
  for (int k = 2; k <= n_pow2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n_pow2; i += blockDim.x) {
        int l = i ^ j;
        if (l > i) {
          bool up = (i & k) == 0;
          int x = a[i], y = a[l];
          if ((x > y) == up) {
            a[i] = y;
            a[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ inline int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
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

struct BuildArgs {
  const int* dom_start;
  const int* bucket;
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
  int* dcol;
  int* dncol;
  int* dp;
  int* dp_count;
  DomainStats* stats;
};

template <int DIM>
__global__ __launch_bounds__(kBuild) void k_dom_build(BuildArgs a) {
  constexpr int REC = DIM == 2 ? 4 : 12;
  __shared__ int s_cid[CD_MAX_DC];
  __shared__ int s_ep[CD_MAX_DP];
  __shared__ int s_pos[CD_MAX_DC];
  __shared__ unsigned long long s_mask[CD_MAX_DP];
  __shared__ short s_col[CD_MAX_DC];
  __shared__ int s_coloff[CD_MAX_COLORS + 1];
  __shared__ int s_np, s_ncol, s_bad;

  const int d = blockIdx.x;
  const int cs = a.dom_start[d], ce = a.dom_start[d + 1];
  const int nct = ce - cs;
  if (threadIdx.x == 0) s_bad = 0;
  if (nct > CD_MAX_DC) {
    if (threadIdx.x == 0) atomicMax(&a.stats->overflow, 1);
    return;
  }
  // 1. the domain's contacts in canonical order
  const int pc = pow2_at_least(nct > 0 ? nct : 1);
  for (int k = threadIdx.x; k < pc; k += blockDim.x) s_cid[k] = k < nct ? a.bucket[cs + k] : 0x7fffffff;
  __syncthreads();
  bitonic_sort(s_cid, pc);
  // 2. its particles: sorted unique finite-mass endpoints
  const int ne = 2 * nct;
  const int pe = pow2_at_least(ne > 0 ? ne : 1);
  for (int k = threadIdx.x; k < pe; k += blockDim.x) {
    int v = 0x7fffffff;
    if (k < ne) {
      int c = s_cid[k >> 1];
      int b = (k & 1) ? a.cj[c] : a.ci[c];
      if (b < a.n) v = b;
    }
    s_ep[k] = v;
  }
  __syncthreads();
  bitonic_sort(s_ep, pe);
  if (threadIdx.x == 0) {
    // compact in place (serial; at most 2 CD_MAX_DC entries)
    int np = 0;
    for (int k = 0; k < ne; ++k) {
      int v = s_ep[k];
      if (v == 0x7fffffff) break;
      if (np == 0 || s_ep[np - 1] != v) s_ep[np++] = v;
    }
    s_np = np;
  }
  __syncthreads();
  const int np = s_np;
  for (int k = threadIdx.x; k < np; k += blockDim.x) s_mask[k] = 0ull;
  __syncthreads();
  // 3. greedy first-fit colouring in canonical order (serial by design)
  if (threadIdx.x == 0) {
    int ncol = 0;
    for (int k = 0; k < nct; ++k) {
      int c = s_cid[k];
      int la = lower_bound_i(s_ep, np, a.ci[c]);
      int bj = a.cj[c];
      int lb = bj < a.n ? lower_bound_i(s_ep, np, bj) : -1;
      unsigned long long used = s_mask[la] | (lb >= 0 ? s_mask[lb] : 0ull);
      if (used == ~0ull) {
        s_bad = 1;
        break;
      }
      int col = __ffsll((long long)~used) - 1;
      s_col[k] = (short)col;
      s_mask[la] |= 1ull << col;
      if (lb >= 0) s_mask[lb] |= 1ull << col;
      if (col + 1 > ncol) ncol = col + 1;
    }
    // stable counting sort by colour
    for (int q = 0; q <= CD_MAX_COLORS; ++q) s_coloff[q] = 0;
    if (!s_bad) {
      for (int k = 0; k < nct; ++k) s_coloff[s_col[k] + 1] += 1;
      for (int q = 0; q < ncol; ++q) s_coloff[q + 1] += s_coloff[q];
      int run[CD_MAX_COLORS];
      for (int q = 0; q < ncol; ++q) run[q] = s_coloff[q];
      for (int k = 0; k < nct; ++k) s_pos[k] = run[s_col[k]]++;
    }
    s_ncol = ncol;
  }
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0) atomicMax(&a.stats->overflow, 2);
    return;
  }
  const int ncol = s_ncol;
  if (threadIdx.x == 0) {
    atomicMax(&a.stats->max_colors, ncol);
    atomicMax(&a.stats->max_contacts, nct);
    atomicMax(&a.stats->max_particles, np);
    a.dncol[d] = ncol;
  }
  for (int q = threadIdx.x; q <= CD_MAX_COLORS; q += blockDim.x)
    a.dcol[(int64_t)d * (CD_MAX_COLORS + 1) + q] = q <= ncol ? s_coloff[q] : nct;
  const int64_t dp0 = 2 * (int64_t)cs;
  for (int k = threadIdx.x; k < np; k += blockDim.x) a.dp[dp0 + k] = s_ep[k];
  if (threadIdx.x == 0) a.dp_count[d] = np;
  // 4. slot arrays
  const int64_t nc = a.nc, cap = a.cap, nn = a.n;
  for (int k = threadIdx.x; k < nct; k += blockDim.x) {
    const int c = s_cid[k];
    const int64_t s = cs + s_pos[k];
    const int i = a.ci[c], j = a.cj[c];
    a.slot_contact[s] = c;
    a.contact_slot[c] = (int)s;
    a.color[c] = s_col[k];
    int la = lower_bound_i(s_ep, np, i);
    int lb = j < nn ? lower_bound_i(s_ep, np, j) : -1 - (int)(j - nn);
    a.ab[s] = make_int2(la, lb);
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
      rc[0] = rn;
      rc[1] = r1;
      rc[2] = r2;
      rc[3] = 0.0;
      for (int q = 0; q < 3; ++q) {
        double fq = rn * n3[q] + r1 * t1[q];
        rc[4 + q] = fq + r2 * t2[q];
        rc[8 + q] = r1 * t2[q] - r2 * t1[q];
      }
      rc[7] = 0.0;
      rc[11] = 0.0;
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

// sort each particle's incidences by contact id, then refer to slots
__global__ __launch_bounds__(kThreads) void k_inc_finish(int64_t n, const int* ptr,
                                                        const int* contact_slot, int* inc) {
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
  for (int k = s0; k < s1; ++k) {
    int v = inc[k];
    inc[k] = 2 * contact_slot[v >> 1] + (v & 1);
  }
}

}  // namespace

hipError_t cd_launch_order(cd_ctx* c) {
  const int64_t nc = c->nc;
  const int P = c->P;
  hipError_t e;
  e = hipMemsetAsync(c->dom_count, 0, sizeof(int) * (size_t)(P + 1), c->stream);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(c->d_stats, 0, sizeof(DomainStats), c->stream);
  if (e != hipSuccess) return e;
  if (nc > 0)
    hipLaunchKernelGGL(k_dom_count, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->dom, nc, c->dom_count);
  e = cd_scan_exclusive(c, c->dom_count, c->dom_start, P);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(c->dom_cursor, 0, sizeof(int) * (size_t)(P + 1), c->stream);
  if (e != hipSuccess) return e;
  if (nc > 0)
    hipLaunchKernelGGL(k_dom_scatter, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->dom, nc, c->dom_start, c->dom_cursor, c->bucket);
  BuildArgs a;
  a.dom_start = c->dom_start;
  a.bucket = c->bucket;
  a.ci = c->ci;
  a.cj = c->cj;
  a.nrm = c->nrm;
  a.gap = c->gap;
  a.R = c->R;
  a.r = c->r;
  a.inv_m = c->inv_m;
  a.inv_I = c->inv_I;
  a.n = c->n;
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
  a.dcol = c->dcol;
  a.dncol = c->dncol;
  a.dp = c->dp;
  a.dp_count = c->dp_count;
  a.stats = c->d_stats;
  if (c->dim == 2)
    hipLaunchKernelGGL(k_dom_build<2>, dim3(P), dim3(kBuild), 0, c->stream, a);
  else
    hipLaunchKernelGGL(k_dom_build<3>, dim3(P), dim3(kBuild), 0, c->stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // incidence lists
  e = hipMemsetAsync(c->inc_count, 0, sizeof(int) * (size_t)(c->n + 1), c->stream);
  if (e != hipSuccess) return e;
  if (nc > 0)
    hipLaunchKernelGGL(k_inc_count, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->ci, c->cj, nc, c->n, c->inc_count);
  e = cd_scan_exclusive(c, c->inc_count, c->inc_ptr, c->n);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(c->inc_cursor, 0, sizeof(int) * (size_t)(c->n + 1), c->stream);
  if (e != hipSuccess) return e;
  if (nc > 0)
    hipLaunchKernelGGL(k_inc_fill, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->ci, c->cj, nc, c->n, c->inc_ptr, c->inc_cursor, c->inc);
  hipLaunchKernelGGL(k_inc_finish, dim3(cd_blocks(c->n, kThreads)), dim3(kThreads), 0, c->stream,
                     c->n, c->inc_ptr, c->contact_slot, c->inc);
  return hipGetLastError();
}
