// update.hip - per-particle derived constants and the semi-implicit Euler
// step (Eqs. 1-2 and the rotational analogue): the new velocity is the old
// one plus dt/m times the external force and every contact force of the
// final sweep (summed in ascending contact id), and the position moves with
// the new velocity.
#include "cd_internal.h"

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_derived(const double* m, const double* inertia,
                                                     int64_t n, double dt, double* inv_m,
                                                     double* inv_I, double* dtim, double* dtii) {
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  double im = 1.0 / m[i], ii = 1.0 / inertia[i];
  inv_m[i] = im;
  inv_I[i] = ii;
  dtim[i] = dt * im;
  dtii[i] = dt * ii;
}

// periodic axes (length > 0) and the box's lower corner
struct Period {
  double lo[3], len[3];
};

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_update(double* x, double* v, double* w,
                                                    const double* f, const double* t,
                                                    const double* r, const double* dtim,
                                                    const double* dtii, const int* inc_ptr,
                                                    const int* inc, const double* rec,
                                                    int64_t n, double dt,
                                                    Period per) {
  constexpr int DR = DIM == 2 ? 1 : 3;
  constexpr int REC = cd_rec(DIM);
  int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  double acc[DIM], tacc[DR];
  for (int k = 0; k < DIM; ++k) acc[k] = f[k * n + p];
  for (int k = 0; k < DR; ++k) tacc[k] = t[k * n + p];
  const double rp = r[p];
  for (int e = inc_ptr[p]; e < inc_ptr[p + 1]; ++e) {
    const int ent = inc[e];
    const double* rc = rec + (int64_t)(ent >> 1) * REC;
    if (DIM == 2) {
      double F0 = rc[2], F1 = rc[3], q = rc[1];
      if (ent & 1) {
        acc[0] = acc[0] + F0;
        acc[1] = acc[1] + F1;
      } else {
        acc[0] = acc[0] - F0;
        acc[1] = acc[1] - F1;
      }
      tacc[0] = tacc[0] - rp * q;
    } else {
      double F[3], Q[3];
      cd_record_force3(rec, ent >> 1, F, Q);
      for (int k = 0; k < 3; ++k) acc[k] = (ent & 1) ? acc[k] + F[k] : acc[k] - F[k];
      for (int k = 0; k < 3; ++k) tacc[k] = tacc[k] - rp * Q[k];
    }
  }
  const double dm = dtim[p], di = dtii[p];
  for (int k = 0; k < DIM; ++k) {
    double V = v[k * n + p] + dm * acc[k];
    v[k * n + p] = V;
    double q = x[k * n + p] + V * dt;
    // a particle leaving a periodic box enters it on the other side
    if (per.len[k] > 0.0) {
      const double L = per.len[k], lo = per.lo[k];
      if (q >= lo + L) q = q - L;
      else if (q < lo) q = q + L;
    }
    x[k * n + p] = q;
  }
  for (int k = 0; k < DR; ++k) w[k * n + p] = w[k * n + p] + di * tacc[k];
}

// Contacts that carry a force after the solve (R_n > 0: closed contacts)
// and those of them at the Coulomb bound (sliding, Eqs. 8-9: the projection
// sets |R_t| to mu R_n, exactly in 2D and up to the rounding of the scaled
// components in 3D), summed per block and added to count[1] and count[0].
// mu_slot (per-slot friction of the solve) with contact_slot, or the shared
// coefficient *mu.
__global__ __launch_bounds__(kThreads) void k_count_active(int dim, const double* R, int64_t nc,
                                                          const double* mu_slot,
                                                          const int* contact_slot,
                                                          const double* mu,
                                                          unsigned long long* count) {
  __shared__ int part[2][kThreads / 64];
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int on = 0, slide = 0;
  if (c < nc && R[c] > 0.0) {
    on = 1;
    const double m = mu_slot ? mu_slot[contact_slot[c]] : *mu;
    const double lim = m * R[c];
    if (dim == 2) {
      slide = fabs(R[nc + c]) == lim ? 1 : 0;
    } else {
      const double t1 = R[nc + c], t2 = R[2 * nc + c];
      slide = t1 * t1 + t2 * t2 >= (lim * lim) * (1.0 - 1e-12) ? 1 : 0;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    on += __shfl_xor(on, off, 64);
    slide += __shfl_xor(slide, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = slide;
    part[1][threadIdx.x >> 6] = on;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    int s = 0;
    for (int k = 0; k < kThreads / 64; ++k) s += part[threadIdx.x][k];
    if (s) atomicAdd(count + threadIdx.x, (unsigned long long)s);
  }
}

// Velocity of each wall after the final forces (Eq. 1 for the wall body): a
// wall of finite mass takes u_n + dt/M (F - sum of R_n over its contacts in
// ascending contact id) along its normal nu and keeps its tangential
// velocity; the others keep theirs.  One workgroup per wall: the forces are
// read in parallel into LDS and summed in order by one thread.
__global__ __launch_bounds__(kThreads) void k_wall_velocities(int dim, int W, int mobile,
                                                             const double* wall,
                                                             const double* rec, int REC,
                                                             const int* wall_slot,
                                                             const int* wall_cnt, int64_t cap,
                                                             double* out) {
  __shared__ double buf[kThreads];
  const int q = blockIdx.x;
  const double* nu = wall + q * dim;
  const double* u = wall + W * dim + W + q * dim;
  if (!((mobile >> q) & 1)) {
    if (threadIdx.x < dim) out[q * dim + threadIdx.x] = u[threadIdx.x];
    return;
  }
  const int cnt = wall_cnt[q];
  const int* ls = wall_slot + (int64_t)q * cap;
  double acc = wall[CD_WALL_FORCE + q];
  for (int base = 0; base < cnt; base += kThreads) {
    const int k = base + threadIdx.x;
    if (k < cnt) buf[threadIdx.x] = rec[(int64_t)ls[k] * REC];
    __syncthreads();
    if (threadIdx.x == 0) {
      const int m = cnt - base < kThreads ? cnt - base : kThreads;
      for (int e = 0; e < m; ++e) acc = acc - buf[e];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double un = 0.0;
    for (int k = 0; k < dim; ++k) un = un + nu[k] * u[k];
    const double un1 = un + wall[CD_WALL_DTIM + q] * acc;
    for (int k = 0; k < dim; ++k) out[q * dim + k] = (u[k] - un * nu[k]) + un1 * nu[k];
  }
}

}  // namespace

hipError_t cd_launch_wall_velocities(cd_ctx* c) {
  if (c->W == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wall_velocities, dim3(c->W), dim3(kThreads), 0, c->stream, c->dim, c->W,
                     c->mobile_mask, c->d_wall, c->rec[c->h_state->iter & 1],
                     cd_rec(c->dim), c->wall_slot, c->wall_cnt, c->cap, c->d_wall_new);
  return hipGetLastError();
}

hipError_t cd_launch_count_active(cd_ctx* c, unsigned long long* count) {
  hipError_t e = hipMemsetAsync(count, 0, 2 * sizeof(unsigned long long), c->stream);
  if (e != hipSuccess || c->nc == 0) return e;
  hipLaunchKernelGGL(k_count_active, dim3(cd_blocks(c->nc, kThreads)), dim3(kThreads), 0,
                     c->stream, c->dim, c->R, c->nc, c->use_mu_slot ? c->mu_slot : nullptr,
                     c->contact_slot, c->d_wall + CD_WALL_MU, count);
  return hipGetLastError();
}

hipError_t cd_launch_derived(cd_ctx* c) {
  hipLaunchKernelGGL(k_derived, dim3(cd_blocks(c->n, kThreads)), dim3(kThreads), 0, c->stream,
                     c->m, c->I, c->n, c->p.dt, c->inv_m, c->inv_I, c->dtim, c->dtii);
  return hipGetLastError();
}

hipError_t cd_launch_update(cd_ctx* c, int final_iter) {
  const double* rec = c->rec[final_iter & 1];
  int nb = cd_blocks(c->n, kThreads);
  Period per;
  for (int k = 0; k < 3; ++k) {
    per.lo[k] = c->lo[k];
    per.len[k] = k < c->dim ? c->period[k] : 0.0;
  }
  if (c->dim == 2)
    hipLaunchKernelGGL(k_update<2>, dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->v, c->w, c->f,
                       c->t, c->r, c->dtim, c->dtii, c->inc_ptr, c->inc, rec, c->n,
                       c->p.dt, per);
  else
    hipLaunchKernelGGL(k_update<3>, dim3(nb), dim3(kThreads), 0, c->stream, c->x, c->v, c->w, c->f,
                       c->t, c->r, c->dtim, c->dtii, c->inc_ptr, c->inc, rec, c->n,
                       c->p.dt, per);
  return hipGetLastError();
}
