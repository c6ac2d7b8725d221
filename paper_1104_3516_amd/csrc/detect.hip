// detect.hip - boundary width, cell binning and pair search into the
// canonical contact list, per-contact geometry and the warm start.
//
// Candidate contacts are the particle pairs and particle-wall pairs whose
// gap is <= skin = 2 vmax dt: two bodies can only touch within the step if
// their gap is below the distance they can close (Sec. 3.1, boundary width).
// The cell grid has a mesh >= 2.2 r_max (Sec. 3.2), so partners lie in the
// 3^dim neighbouring cells.  The list is written directly in canonical
// (i, j) order: particle i owns a contiguous range found by a prefix sum of
// its pair count, sorted by j, walls last.
#include "cd_internal.h"

namespace {

constexpr int kThreads = 256;

__device__ inline void atomic_max_nonneg(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_vmax(const double* v, int64_t n,
                                                  unsigned long long* out) {
  __shared__ double sh[kThreads / 64];
  double best = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double q = v[i] * v[i];
    q = q + v[n + i] * v[n + i];
    if (DIM == 3) q = q + v[2 * n + i] * v[2 * n + i];
    double s = sqrt(q);
    // a NaN speed must win the maximum so that it is reported
    if (s > best || s != s) best = s;
  }
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(best, off, 64);
    if (o > best || o != o) best = o;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sh[0];
    for (int k = 1; k < kThreads / 64; ++k)
      if (sh[k] > b || sh[k] != sh[k]) b = sh[k];
    atomic_max_nonneg(out, b != b ? __longlong_as_double(0x7ff8000000000000ll) : b);
  }
}

struct CellGrid {
  double lo[3];
  double width[3];
  double period[3];   // > 0: periodic axis of this length (the box's)
  int ncell[3];
};

// Separation along a periodic axis of length L: the nearest image.
__device__ inline double min_image(double d, double L) {
  if (d > 0.5 * L) return d - L;
  if (d < -0.5 * L) return d + L;
  return d;
}

// A coordinate back into [lo, lo + L) after it left by less than L.
__device__ inline double wrap_into(double q, double lo, double L) {
  if (q >= lo + L) return q - L;
  if (q < lo) return q + L;
  return q;
}

template <int DIM>
__device__ inline int cell_coord(double x, double lo, double width, int ncell) {
  double q = floor((x - lo) / width);
  if (q < 0.0) return 0;
  if (q > (double)(ncell - 1)) return ncell - 1;
  return (int)q;
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_cell_bin(const double* x, int64_t n, CellGrid g,
                                                      int* cell_of, int* cell_count) {
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  int c0 = cell_coord<DIM>(x[i], g.lo[0], g.width[0], g.ncell[0]);
  int c1 = cell_coord<DIM>(x[n + i], g.lo[1], g.width[1], g.ncell[1]);
  int c2 = DIM == 3 ? cell_coord<DIM>(x[2 * n + i], g.lo[2], g.width[2], g.ncell[2]) : 0;
  int cell = (c2 * g.ncell[1] + c1) * g.ncell[0] + c0;
  cell_of[i] = cell;
  atomicAdd(&cell_count[cell], 1);
}

// Each particle's place in its cell's member list, with a copy of its
// position and radius at the same place (xr, (DIM + 1) x n), so that the
// pair search reads its candidates' data in cell order, without going
// through the member ids first.
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_cell_scatter(int64_t n, const int* cell_of,
                                                          const int* cell_start, int* cursor,
                                                          int* members, const double* x,
                                                          const double* r, double* xr) {
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  int cell = cell_of[i];
  int pos = atomicAdd(&cursor[cell], 1);
  const int64_t s = cell_start[cell] + pos;
  members[s] = (int)i;
  for (int k = 0; k < DIM; ++k) xr[k * n + s] = x[k * n + i];
  xr[DIM * n + s] = r[i];
}

// squared distance of particles i < j at the nearest image along periodic
// axes; their gap (Sec. 2.1, Fig. 1) is its square root minus both radii
template <int DIM>
__device__ inline double pair_dist2(const double* xi, const double* xj, const CellGrid& g) {
  double d0 = xj[0] - xi[0];
  if (g.period[0] > 0.0) d0 = min_image(d0, g.period[0]);
  double d1 = xj[1] - xi[1];
  if (g.period[1] > 0.0) d1 = min_image(d1, g.period[1]);
  double d2 = d0 * d0;
  d2 = d2 + d1 * d1;
  if (DIM == 3) {
    double e = xj[2] - xi[2];
    if (g.period[2] > 0.0) e = min_image(e, g.period[2]);
    d2 = d2 + e * e;
  }
  return d2;
}


// gap of particle i and wall w: (nu.x - o) - r_i
template <int DIM>
__device__ inline double wall_gap(const double* x, const double* r, int64_t n, int i,
                                  const double* wall, int W, int w) {
  const double* nu = wall + w * DIM;
  double proj = 0.0;
  for (int k = 0; k < DIM; ++k) proj = proj + nu[k] * x[k * n + i];
  return (proj - wall[W * DIM + w]) - r[i];
}

// The boundary width of the step: `fixed` when given (>= 0), else 2 vmax dt
// with vmax the larger of the particles' maximum speed (device, from k_vmax)
// and the walls' (host): the same operations as the host's check of it.
struct SkinArgs {
  const unsigned long long* vmax_bits;
  double wall_speed, fixed, dt;
};

__device__ inline double skin_of(const SkinArgs& k) {
  if (k.fixed >= 0.0) return k.fixed;
  double vm = __longlong_as_double((long long)*k.vmax_bits);
  if (k.wall_speed > vm) vm = k.wall_speed;
  return 2.0 * vm * k.dt;
}

template <int DIM, bool FILL>
__global__ __launch_bounds__(kThreads) void k_pairs(const double* x, const double* r, int64_t n,
                                                   CellGrid g, const int* cell_of,
                                                   const int* cell_start, const int* members,
                                                   const double* xr, const double* wall, int W,
                                                   SkinArgs sk, int* count, const int* off,
                                                   int* ci, int* cj) {
  int64_t ii = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (ii >= n) return;
  const double skin = skin_of(sk);
  int i = (int)ii;
  const double ri = r[i];
  double xi[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < DIM; ++k) xi[k] = x[k * n + i];
  int cell = cell_of[i];
  int cx = cell % g.ncell[0];
  int cy = (cell / g.ncell[0]) % g.ncell[1];
  int cz = cell / (g.ncell[0] * g.ncell[1]);
  int k = 0;
  int base = FILL ? off[i] : 0;
  const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
  // along a periodic axis (three cells at least) the neighbour cells wrap
  for (int dz = zlo; dz <= zhi; ++dz) {
    int qz = cz + dz;
    if (DIM == 3 && g.period[2] > 0.0) qz = (qz + g.ncell[2]) % g.ncell[2];
    if (qz < 0 || qz >= g.ncell[2]) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int qy = cy + dy;
      if (g.period[1] > 0.0) qy = (qy + g.ncell[1]) % g.ncell[1];
      if (qy < 0 || qy >= g.ncell[1]) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        int qx = cx + dx;
        if (g.period[0] > 0.0) qx = (qx + g.ncell[0]) % g.ncell[0];
        if (qx < 0 || qx >= g.ncell[0]) continue;
        int q = (qz * g.ncell[1] + qy) * g.ncell[0] + qx;
        for (int s = cell_start[q]; s < cell_start[q + 1]; ++s) {
          // the candidate's position and radius in cell order (the same
          // values as x[j], r[j])
          double xj[3] = {0.0, 0.0, 0.0};
          for (int k = 0; k < DIM; ++k) xj[k] = xr[k * n + s];
          const double rj = xr[DIM * n + s];
          int j = members[s];
          if (j <= i) continue;
          // a pair whose squared distance exceeds (r_i + r_j + skin)^2 by a
          // relative margin of 2e-9 cannot pass the test below, whatever the
          // rounding (its errors are some 1e-15 relative): no square root
          const double d2 = pair_dist2<DIM>(xi, xj, g);
          const double reach = ((ri + rj) + skin) * (1.0 + 1e-9);
          if (d2 > reach * reach) continue;
          if ((sqrt(d2) - ri) - rj <= skin) {
            if (FILL) {
              // insertion into the particle's sorted range
              int pos = k;
              while (pos > 0 && cj[base + pos - 1] > j) {
                cj[base + pos] = cj[base + pos - 1];
                --pos;
              }
              cj[base + pos] = j;
              ci[base + k] = i;
            }
            ++k;
          }
        }
      }
    }
  }
  for (int w = 0; w < W; ++w) {
    if (wall_gap<DIM>(x, r, n, i, wall, W, w) <= skin) {
      if (FILL) {
        ci[base + k] = i;
        cj[base + k] = (int)n + w;
      }
      ++k;
    }
  }
  if (!FILL) count[i] = k;
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_geometry(const double* x, const double* r, int64_t n,
                                                      const double* wall, int W, int64_t nc,
                                                      const int* ci, const int* cj, double* nrm,
                                                      double* gap, double* xmid, CellGrid gr) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  int i = ci[c], j = cj[c];
  double nv[3] = {0.0, 0.0, 0.0};
  double g;
  if (j < n) {
    double d[3] = {0.0, 0.0, 0.0};
    double d2 = 0.0;
    for (int k = 0; k < DIM; ++k) {
      d[k] = x[k * n + j] - x[k * n + i];
      if (gr.period[k] > 0.0) d[k] = min_image(d[k], gr.period[k]);
      d2 = d2 + d[k] * d[k];
    }
    double dist = sqrt(d2);
    for (int k = 0; k < DIM; ++k) nv[k] = d[k] / dist;
    g = (dist - r[i]) - r[j];
  } else {
    int w = j - (int)n;
    const double* nu = wall + w * DIM;
    double proj = 0.0;
    for (int k = 0; k < DIM; ++k) proj = proj + nu[k] * x[k * n + i];
    for (int k = 0; k < DIM; ++k) nv[k] = -nu[k];
    g = (proj - wall[W * DIM + w]) - r[i];
  }
  gap[c] = g;
  // contact position: the middle of the gap (Sec. 3.1)
  double lever = r[i] + 0.5 * g;
  for (int k = 0; k < DIM; ++k) {
    nrm[k * nc + c] = nv[k];
    double q = x[k * n + i] + lever * nv[k];
    // on a periodic axis the contact position is taken back into the box
    if (gr.period[k] > 0.0) q = wrap_into(q, gr.lo[k], gr.period[k]);
    xmid[k * nc + c] = q;
  }
}

// start from the previous step's force of the same pair, else zero
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_warm(int64_t nc, const int* ci, const int* cj,
                                                  int64_t nprev, const int* pi, const int* pj,
                                                  const double* Rprev, double* R) {
  int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= nc) return;
  int a = ci[c], b = cj[c];
  int64_t lo = 0, hi = nprev;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (pi[mid] < a || (pi[mid] == a && pj[mid] < b)) lo = mid + 1;
    else hi = mid;
  }
  bool found = lo < nprev && pi[lo] == a && pj[lo] == b;
  for (int k = 0; k < DIM; ++k) R[k * nc + c] = found ? Rprev[k * nprev + lo] : 0.0;
}

}  // namespace

hipError_t cd_launch_vmax(cd_ctx* c) {
  hipError_t e = hipMemsetAsync(c->d_vmax, 0, sizeof(unsigned long long), c->stream);
  if (e != hipSuccess) return e;
  int nb = cd_blocks(c->n, kThreads);
  if (nb > 1024) nb = 1024;
  if (c->dim == 2)
    hipLaunchKernelGGL(k_vmax<2>, dim3(nb), dim3(kThreads), 0, c->stream, c->v, c->n, c->d_vmax);
  else
    hipLaunchKernelGGL(k_vmax<3>, dim3(nb), dim3(kThreads), 0, c->stream, c->v, c->n, c->d_vmax);
  return hipGetLastError();
}

static CellGrid make_grid(cd_ctx* c) {
  CellGrid g;
  for (int k = 0; k < 3; ++k) {
    g.lo[k] = c->lo[k];
    g.width[k] = c->cwidth[k];
    g.ncell[k] = c->ncell[k];
    g.period[k] = k < c->dim ? c->period[k] : 0.0;
  }
  return g;
}

hipError_t cd_launch_cells(cd_ctx* c) {
  hipError_t e = hipMemsetAsync(c->cell_count, 0, sizeof(int) * (size_t)(c->ncells + 1), c->stream);
  if (e != hipSuccess) return e;
  CellGrid g = make_grid(c);
  int nb = cd_blocks(c->n, kThreads);
  if (c->dim == 2)
    hipLaunchKernelGGL(k_cell_bin<2>, dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->n, g,
                       c->cell_of, c->cell_count);
  else
    hipLaunchKernelGGL(k_cell_bin<3>, dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->n, g,
                       c->cell_of, c->cell_count);
  e = cd_scan_exclusive(c, c->cell_count, c->cell_start, c->ncells);
  if (e != hipSuccess) return e;
  // reuse cell_count as the scatter cursor
  e = hipMemsetAsync(c->cell_count, 0, sizeof(int) * (size_t)(c->ncells + 1), c->stream);
  if (e != hipSuccess) return e;
  if (c->dim == 2)
    hipLaunchKernelGGL(k_cell_scatter<2>, dim3(nb), dim3(kThreads), 0, c->stream, c->n,
                       c->cell_of, c->cell_start, c->cell_count, c->cell_members, c->x, c->r,
                       c->cell_xr);
  else
    hipLaunchKernelGGL(k_cell_scatter<3>, dim3(nb), dim3(kThreads), 0, c->stream, c->n,
                       c->cell_of, c->cell_start, c->cell_count, c->cell_members, c->x, c->r,
                       c->cell_xr);
  return hipGetLastError();
}

hipError_t cd_launch_pair_count(cd_ctx* c) {
  CellGrid g = make_grid(c);
  const SkinArgs skin{c->d_vmax, c->st_wall_speed, c->p.skin, c->p.dt};
  int nb = cd_blocks(c->n, kThreads);
  if (c->dim == 2)
    hipLaunchKernelGGL((k_pairs<2, false>), dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->r,
                       c->n, g, c->cell_of, c->cell_start, c->cell_members, c->cell_xr, c->d_wall, c->W,
                       skin,
                       c->pair_count, nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_pairs<3, false>), dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->r,
                       c->n, g, c->cell_of, c->cell_start, c->cell_members, c->cell_xr, c->d_wall, c->W,
                       skin,
                       c->pair_count, nullptr, nullptr, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return cd_scan_exclusive(c, c->pair_count, c->pair_off, c->n);
}

hipError_t cd_launch_pair_fill(cd_ctx* c) {
  CellGrid g = make_grid(c);
  const SkinArgs skin{c->d_vmax, c->st_wall_speed, c->p.skin, c->p.dt};
  int nb = cd_blocks(c->n, kThreads);
  if (c->dim == 2)
    hipLaunchKernelGGL((k_pairs<2, true>), dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->r,
                       c->n, g, c->cell_of, c->cell_start, c->cell_members, c->cell_xr, c->d_wall, c->W,
                       skin,
                       nullptr, c->pair_off, c->ci, c->cj);
  else
    hipLaunchKernelGGL((k_pairs<3, true>), dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->r,
                       c->n, g, c->cell_of, c->cell_start, c->cell_members, c->cell_xr, c->d_wall, c->W,
                       skin,
                       nullptr, c->pair_off, c->ci, c->cj);
  return hipGetLastError();
}

hipError_t cd_launch_geometry(cd_ctx* c) {
  if (c->nc == 0) return hipSuccess;
  int nb = cd_blocks(c->nc, kThreads);
  if (c->dim == 2)
    hipLaunchKernelGGL(k_geometry<2>, dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->r, c->n,
                       c->d_wall, c->W, c->nc, c->ci, c->cj, c->nrm, c->gap, c->xmid,
                       make_grid(c));
  else
    hipLaunchKernelGGL(k_geometry<3>, dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->r, c->n,
                       c->d_wall, c->W, c->nc, c->ci, c->cj, c->nrm, c->gap, c->xmid,
                       make_grid(c));
  return hipGetLastError();
}

hipError_t cd_launch_warm_start(cd_ctx* c) {
  if (c->nc == 0) return hipSuccess;
  int nb = cd_blocks(c->nc, kThreads);
  int64_t nprev = (c->p.warm_start && c->R_prev) ? c->nc_prev : 0;
  if (c->dim == 2)
    hipLaunchKernelGGL(k_warm<2>, dim3(nb), dim3(kThreads), 0, c->stream, c->nc, c->ci, c->cj,
                       nprev, c->ci_prev, c->cj_prev, c->R_prev, c->R);
  else
    hipLaunchKernelGGL(k_warm<3>, dim3(nb), dim3(kThreads), 0, c->stream, c->nc, c->ci, c->cj,
                       nprev, c->ci_prev, c->cj_prev, c->R_prev, c->R);
  return hipGetLastError();
}
