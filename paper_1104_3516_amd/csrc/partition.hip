// partition.hip - hierarchical bisection of the contacts into P domains.
//
// Tree shape (Sec. 3.2, Fig. 8): starting from one node, every node of a
// level is branched until 2^l < P <= 2^(l+1); then only the first P - 2^l
// nodes of level l are branched, left to right.  Leaves are numbered left to
// right and are the domains.
//
// Cuts: each inner node is cut perpendicular to the longest side of its
// region (the shortest interface).  The left branch receives a share of the
// node's contacts proportional to its leaf count: with n contacts and leaf
// counts (L, R) the cut is the k-th smallest contact position on the axis,
// k = floor(n L / (L + R)), and contacts strictly below the cut go left.  A
// node without contacts is cut in the middle of its region.  This balances
// by contact number, the balancing the paper calls the most exact (Sec. 5).
// With per-domain capacities (adaptive load balancing, Sec. 3.3) the left
// branch's share is nu_L / (nu_L + nu_R) instead, nu summing the capacities
// of the leaves below: k = floor(n share), at most n - 1.
//
// GPU form: the contact positions are sorted once per axis (stable radix
// sort of order-preserving keys); every node owns one contiguous segment of
// each sorted list.  A level then needs, per node, one read of the k-th
// element and one binary search, and per list one stable split of every
// segment (flag, prefix sum, scatter).
#include "cd_internal.h"

#include <cmath>

namespace {

constexpr int kThreads = 256;

__device__ inline unsigned long long order_key(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(kThreads) void k_keys(const double* xmid, int64_t nc, int axis,
                                                  unsigned long long* keys, int* vals) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  keys[c] = order_key(xmid[axis * nc + c]);
  vals[c] = (int)c;
}

__global__ void k_root(int* seg_start, int* seg_end, double* region, const double* box, int nc) {
  seg_start[0] = 0;
  seg_end[0] = nc;
  for (int k = 0; k < 6; ++k) region[k] = box[k];
}

__global__ __launch_bounds__(kThreads) void k_fill_int(int* a, int64_t n, int v) {
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) a[i] = v;
}

struct LevelArgs {
  const double* xmid;
  int64_t nc;
  int dim;
  int first, count;
  const int* child;
  const int* leaves;
  const double* frac;   // left-branch shares (capacities), or null: leaf counts
  const int* perm0;
  const int* perm1;
  const int* perm2;
  int* axis;
  double* cut;
  int* nl;
  int* seg_start;
  int* seg_end;
  double* region;
};

__global__ __launch_bounds__(kThreads) void k_level_nodes(LevelArgs a) {
  int q = blockIdx.x * kThreads + threadIdx.x;
  if (q >= a.count) return;
  int node = a.first + q;
  int left = a.child[2 * node], right = a.child[2 * node + 1];
  if (left < 0) return;
  const double* lo = a.region + 6 * node;
  const double* hi = lo + 3;
  int axis = 0;
  double best = hi[0] - lo[0];
  for (int k = 1; k < a.dim; ++k) {
    if (hi[k] - lo[k] > best) {
      best = hi[k] - lo[k];
      axis = k;
    }
  }
  const int* perm = axis == 0 ? a.perm0 : (axis == 1 ? a.perm1 : a.perm2);
  int s0 = a.seg_start[node], s1 = a.seg_end[node];
  long long cnt = s1 - s0;
  long long ll = a.leaves[left], lr = a.leaves[right];
  const double* coord = a.xmid + (int64_t)axis * a.nc;
  double cut;
  int nl = 0;
  if (cnt > 0) {
    long long k;
    if (a.frac) {
      k = (long long)floor((double)cnt * a.frac[node]);
      if (k > cnt - 1) k = cnt - 1;
      if (k < 0) k = 0;
    } else {
      k = (cnt * ll) / (ll + lr);
    }
    cut = coord[perm[s0 + k]];
    // contacts strictly below the cut: first sorted position with coord >= cut
    int lo_i = s0, hi_i = s0 + (int)k;
    while (lo_i < hi_i) {
      int mid = (lo_i + hi_i) >> 1;
      if (coord[perm[mid]] < cut) lo_i = mid + 1;
      else hi_i = mid;
    }
    nl = lo_i - s0;
  } else {
    cut = 0.5 * (lo[axis] + hi[axis]);
  }
  a.axis[node] = axis;
  a.cut[node] = cut;
  a.nl[node] = nl;
  a.seg_start[left] = s0;
  a.seg_end[left] = s0 + nl;
  a.seg_start[right] = s0 + nl;
  a.seg_end[right] = s1;
  double* rl = a.region + 6 * left;
  double* rr = a.region + 6 * right;
  for (int k = 0; k < 6; ++k) {
    rl[k] = lo[k];
    rr[k] = lo[k];
  }
  rl[3 + axis] = cut;   // left: [lo, cut]
  rr[axis] = cut;       // right: [cut, hi]
}

__global__ __launch_bounds__(kThreads) void k_level_side(const double* xmid, int64_t nc, int first,
                                                        int count, const int* child,
                                                        const int* axis, const double* cut,
                                                        int* cnode, int* side) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  int node = cnode[c];
  int s = 0;
  if (node >= first && node < first + count && child[2 * node] >= 0) {
    int a = axis[node];
    s = xmid[(int64_t)a * nc + c] < cut[node] ? 0 : 1;
    cnode[c] = child[2 * node + s];
  }
  side[c] = s;
}

__global__ __launch_bounds__(kThreads) void k_level_flags(const int* perm, const int* side,
                                                         int64_t nc, int* flag) {
  int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q < nc) flag[q] = side[perm[q]];
}

__global__ __launch_bounds__(kThreads) void k_level_scatter(const int* perm, const int* side,
                                                           const int* cnode, const int* parent,
                                                           int first, int count,
                                                           const int* seg_start, const int* nl,
                                                           const int* flag_scan, int64_t nc,
                                                           int* out) {
  int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= nc) return;
  int c = perm[q];
  int node = cnode[c];
  int par = parent[node];
  int64_t pos = q;
  if (par >= first && par < first + count) {
    int s0 = seg_start[par];
    int right_before = flag_scan[q] - flag_scan[s0];
    if (side[c]) pos = (int64_t)s0 + nl[par] + right_before;
    else pos = (int64_t)s0 + (q - s0 - right_before);
  }
  out[pos] = c;
}

__global__ __launch_bounds__(kThreads) void k_leaf_dom(const int* cnode, const int* leaf,
                                                      int64_t nc, int* dom) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c < nc) dom[c] = leaf[cnode[c]];
}

__global__ __launch_bounds__(kThreads) void k_descend(const double* xmid, int64_t nc,
                                                     const int* axis, const double* cut,
                                                     const int* child, const int* leaf, int* dom) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  int node = 0;
  while (leaf[node] < 0) {
    int a = axis[node];
    node = xmid[(int64_t)a * nc + c] < cut[node] ? child[2 * node] : child[2 * node + 1];
  }
  dom[c] = leaf[node];
}

}  // namespace

// Left-branch shares of the inner nodes from the capacities (Sec. 3.3):
// nu of a node is its leaf's capacity or the sum of its two branches' nu
// (nodes are created after their parents, so reverse creation order is
// bottom-up); capacities that are not positive and finite count as the
// mean of the valid ones, or 1.
static void node_shares(const cd_ctx* c, double* share) {
  const int P = c->P, nodes = 2 * P - 1;
  const std::vector<double>& cap = c->lb_capacity;
  double sum = 0.0;
  int valid = 0;
  for (int i = 0; i < P; ++i)
    if (cap[i] > 0.0 && std::isfinite(cap[i])) {
      sum = sum + cap[i];
      ++valid;
    }
  const double fill = valid > 0 ? sum / (double)valid : 1.0;
  std::vector<double> nu(nodes);
  for (int node = nodes - 1; node >= 0; --node) {
    const int l = c->t_child[2 * node], r = c->t_child[2 * node + 1];
    if (l < 0) {
      const double v = cap[c->t_leaf[node]];
      nu[node] = (v > 0.0 && std::isfinite(v)) ? v : fill;
      share[node] = 0.0;
    } else {
      nu[node] = nu[l] + nu[r];
      share[node] = nu[l] / nu[node];
    }
  }
}

hipError_t cd_launch_orb(cd_ctx* c) {
  const int64_t nc = c->nc;
  const int nodes = 2 * c->P - 1;
  hipError_t e;
  // inner-node axis / cut defaults (leaves keep -1 / 0)
  hipLaunchKernelGGL(k_fill_int, dim3(cd_blocks(nodes, kThreads)), dim3(kThreads), 0, c->stream,
                     c->d_axis, (int64_t)nodes, -1);
  e = hipMemsetAsync(c->d_cut, 0, sizeof(double) * (size_t)nodes, c->stream);
  if (e != hipSuccess) return e;
  if (c->P == 1) {
    if (nc > 0) e = hipMemsetAsync(c->dom, 0, sizeof(int) * (size_t)nc, c->stream);
    return e;
  }
  // sorted contact ids per axis
  for (int k = 0; k < c->dim; ++k) {
    if (nc == 0) break;
    hipLaunchKernelGGL(k_keys, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->xmid, nc, k, c->sort_keys[0], c->sort_vals[0]);
    unsigned long long* ko;
    int* vo;
    e = cd_radix_sort(c, c->sort_keys[0], c->sort_vals[0], c->sort_keys[1], c->sort_vals[1], nc, 64,
                      &ko, &vo);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(c->perm[k], vo, sizeof(int) * (size_t)nc, hipMemcpyDeviceToDevice,
                       c->stream);
    if (e != hipSuccess) return e;
  }
  // root: all contacts, the simulation box
  // (the pinned scratch buffer outlives the asynchronous copy)
  double* box = (double*)c->h_scratch;
  for (int k = 0; k < 3; ++k) {
    box[k] = c->lo[k];
    box[3 + k] = c->hi[k];
  }
  double* d_box = c->d_region + 6 * (size_t)nodes;   // spare slot after the node regions
  e = hipMemcpyAsync(d_box, box, 6 * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, c->stream, c->d_seg_start, c->d_seg_end,
                     c->d_region, d_box, (int)nc);
  if (nc > 0)
    hipLaunchKernelGGL(k_fill_int, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->cnode, nc, 0);
  // capacity shares (adaptive load balancing), staged through pinned memory
  const double* frac = nullptr;
  if ((int)c->lb_capacity.size() == c->P) {
    if (!c->h_frac) {
      e = hipHostMalloc((void**)&c->h_frac, sizeof(double) * (size_t)nodes);
      if (e != hipSuccess) return e;
    }
    if (!c->d_frac) {
      e = hipMalloc((void**)&c->d_frac, sizeof(double) * (size_t)nodes);
      if (e != hipSuccess) return e;
    }
    // the previous rebuild's upload has finished (the host synchronises the
    // stream between the phases of every step)
    node_shares(c, c->h_frac);
    e = hipMemcpyAsync(c->d_frac, c->h_frac, sizeof(double) * (size_t)nodes,
                       hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    frac = c->d_frac;
  }
  for (size_t lev = 0; lev < c->t_level_first.size(); ++lev) {
    int first = c->t_level_first[lev], count = c->t_level_count[lev];
    LevelArgs a;
    a.frac = frac;
    a.xmid = c->xmid;
    a.nc = nc;
    a.dim = c->dim;
    a.first = first;
    a.count = count;
    a.child = c->d_child;
    a.leaves = c->d_leaves;
    a.perm0 = c->perm[0];
    a.perm1 = c->perm[1];
    a.perm2 = c->perm[2] ? c->perm[2] : c->perm[0];
    a.axis = c->d_axis;
    a.cut = c->d_cut;
    a.nl = c->d_nl;
    a.seg_start = c->d_seg_start;
    a.seg_end = c->d_seg_end;
    a.region = c->d_region;
    hipLaunchKernelGGL(k_level_nodes, dim3(cd_blocks(count, kThreads)), dim3(kThreads), 0,
                       c->stream, a);
    if (nc == 0) continue;
    int nb = cd_blocks(nc, kThreads);
    hipLaunchKernelGGL(k_level_side, dim3(nb), dim3(kThreads), 0, c->stream, c->xmid, nc, first,
                       count, c->d_child, c->d_axis, c->d_cut, c->cnode, c->side);
    for (int k = 0; k < c->dim; ++k) {
      hipLaunchKernelGGL(k_level_flags, dim3(nb), dim3(kThreads), 0, c->stream, c->perm[k],
                         c->side, nc, c->flag);
      e = cd_scan_exclusive(c, c->flag, c->flag_scan, nc);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_level_scatter, dim3(nb), dim3(kThreads), 0, c->stream, c->perm[k],
                         c->side, c->cnode, c->d_parent, first, count, c->d_seg_start, c->d_nl,
                         c->flag_scan, nc, c->perm_tmp);
      int* t = c->perm[k];
      c->perm[k] = c->perm_tmp;
      c->perm_tmp = t;
    }
  }
  if (nc > 0)
    hipLaunchKernelGGL(k_leaf_dom, dim3(cd_blocks(nc, kThreads)), dim3(kThreads), 0, c->stream,
                       c->cnode, c->d_leaf, nc, c->dom);
  return hipGetLastError();
}

hipError_t cd_launch_descend(cd_ctx* c) {
  if (c->nc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_descend, dim3(cd_blocks(c->nc, kThreads)), dim3(kThreads), 0, c->stream,
                     c->xmid, c->nc, c->d_axis, c->d_cut, c->d_child, c->d_leaf, c->dom);
  return hipGetLastError();
}
