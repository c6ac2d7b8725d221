// sweep.hip - the domain-wise iterative force solve (Sec. 2.1 and 3.1).
//
// One sweep = one kernel launch; one workgroup per domain.
//  1. Exchange: the workgroup recomputes the velocities of its particles
//     from their base velocities and external forces plus every incident
//     contact force of the previous sweep (own and foreign contacts), into
//     LDS.  This is the per-sweep exchange of boundary contact forces: other
//     domains' forces are read from the previous sweep's record array.
//  2. Sequential update: colours in order; in a colour, lanes update
//     contacts that share no particle, each solving its own force law with
//     all other forces fixed (Eqs. 3-9, Fig. 2) and applying the change to
//     both bodies' LDS velocities.  New forces go to the other record array,
//     so no domain ever sees a force of the current sweep from another
//     domain (foreign contacts stay frozen for the sweep).
//  3. Convergence: every workgroup reduces its contacts' test values; the
//     last workgroup to finish reduces all of them in a fixed order and
//     decides (criterion I or II), advancing the sweep counter.  Later
//     launches of the same solve return at once after the stop decision.
//
// Blocks are mapped to domains so that each of the 8 XCDs (blocks are
// dispatched round-robin over them) works on a contiguous run of domains,
// which are spatial neighbours in the bisection tree and share halo data in
// that XCD's L2.
#include "cd_internal.h"

namespace {

constexpr int kInitThreads = 1024;

__device__ inline void store_rel(long long* p, long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline long long load_rel(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DIM>
__device__ inline void local_force(const double* n, const double* t1, const double* t2, double gdt,
                                   double dwn, double dwt, double kn, double kt, double mu,
                                   double ra, double rb, const double* Va, const double* Wa,
                                   const double* Vb, const double* Wb, const double* Rold,
                                   double* Rnew) {
  double dV[3];
  for (int q = 0; q < DIM; ++q) dV[q] = Vb[q] - Va[q];
  double vn = 0.0;
  for (int q = 0; q < DIM; ++q) vn = vn + dV[q] * n[q];
  double vt1, vt2 = 0.0;
  if (DIM == 2) {
    double dvt = dV[0] * t1[0] + dV[1] * t1[1];
    double spin = ra * Wa[0] + rb * Wb[0];
    vt1 = dvt - spin;
  } else {
    double spin[3];
    for (int q = 0; q < 3; ++q) spin[q] = ra * Wa[q] + rb * Wb[q];
    double dvt1 = 0.0, dvt2 = 0.0, s2 = 0.0, s1 = 0.0;
    for (int q = 0; q < 3; ++q) {
      dvt1 = dvt1 + dV[q] * t1[q];
      dvt2 = dvt2 + dV[q] * t2[q];
      s2 = s2 + spin[q] * t2[q];
      s1 = s1 + spin[q] * t1[q];
    }
    vt1 = dvt1 - s2;
    vt2 = dvt2 + s1;
  }
  // relative velocity the pair would have without this contact's force
  double un = vn - dwn * Rold[0];
  double ut1 = vt1 - dwt * Rold[1];
  double ut2 = DIM == 3 ? vt2 - dwt * Rold[2] : 0.0;
  double s = gdt + un;      // predicted gap / dt (Eq. 3)
  Rnew[0] = 0.0;
  Rnew[1] = 0.0;
  if (DIM == 3) Rnew[2] = 0.0;
  if (s >= 0.0) return;     // stays open
  double rn = -s * kn;      // sticking force, normal part (Eqs. 4-5)
  double T1 = -ut1 * kt;
  double T2 = DIM == 3 ? -ut2 * kt : 0.0;
  double lim = mu * rn;     // Coulomb bound (Eq. 7)
  Rnew[0] = rn;
  if (DIM == 2) {
    if (fabs(T1) <= lim) Rnew[1] = T1;
    else Rnew[1] = T1 > 0.0 ? lim : -lim;   // sliding (Eqs. 8-9)
  } else {
    double tn = sqrt(T1 * T1 + T2 * T2);
    if (tn <= lim) {
      Rnew[1] = T1;
      Rnew[2] = T2;
    } else {
      double fac = lim / tn;
      Rnew[1] = T1 * fac;
      Rnew[2] = T2 * fac;
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
  constexpr int DR = DIM == 2 ? 1 : 3;
  constexpr int REC = DIM == 2 ? 4 : 12;
  extern __shared__ double lds[];
  __shared__ long long sh_np[4];
  __shared__ double sh_md[4], sh_sr[4];
  __shared__ int sh_last;

  SolveState* st = a.state;
  if (*(volatile int*)&st->done) return;
  const int j = *(volatile int*)&st->iter + 1;
  const double* rin = a.rec[(j - 1) & 1];
  double* rout = a.rec[j & 1];
  const int b = blockIdx.x;
  const int d = (b % 8) * a.per_xcd + b / 8;
  const int tid = threadIdx.x, nthr = blockDim.x;

  long long npass = 0;
  double maxd = 0.0, sumr = 0.0;

  if (d < a.P) {
    const int cs = a.dom_start[d];
    const int np = a.dp_count[d];
    const int* dpl = a.dp + 2 * (int64_t)cs;
    const int stride = np;   // LDS arrays are [component][local particle]
    double* sV = lds;
    double* sW = sV + DIM * stride;
    double* sdm = sW + DR * stride;
    double* sdi = sdm + stride;
    double* sr = sdi + stride;
    const int64_t n = a.n;
    // 1. exchange: velocities from the previous sweep's forces
    for (int l = tid; l < np; l += nthr) {
      const int p = dpl[l];
      double acc[DIM], tacc[DR];
      for (int k = 0; k < DIM; ++k) acc[k] = a.f[k * n + p];
      for (int k = 0; k < DR; ++k) tacc[k] = a.t[k * n + p];
      const double rp = a.r[p];
      const int e1 = a.inc_ptr[p + 1];
      for (int e = a.inc_ptr[p]; e < e1; ++e) {
        const int ent = a.inc[e];
        const double* rc = rin + (int64_t)(ent >> 1) * REC;
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
          for (int k = 0; k < 3; ++k) {
            double F = rc[4 + k];
            acc[k] = (ent & 1) ? acc[k] + F : acc[k] - F;
          }
          for (int k = 0; k < 3; ++k) tacc[k] = tacc[k] - rp * rc[8 + k];
        }
      }
      const double dm = a.dtim[p], di = a.dtii[p];
      for (int k = 0; k < DIM; ++k) sV[k * stride + l] = a.v[k * n + p] + dm * acc[k];
      for (int k = 0; k < DR; ++k) sW[k * stride + l] = a.w[k * n + p] + di * tacc[k];
      sdm[l] = dm;
      sdi[l] = di;
      sr[l] = rp;
    }
    __syncthreads();
    // 2. colour-major sequential update
    const int ncol = a.dncol[d];
    const int* co = a.dcol + (int64_t)d * (CD_MAX_COLORS + 1);
    const int64_t cap = a.cap;
    const double* g = a.geo;
    for (int col = 0; col < ncol; ++col) {
      const int s0 = cs + co[col], s1 = cs + co[col + 1];
      for (int s = s0 + tid; s < s1; s += nthr) {
        const int2 ab = a.ab[s];
        double nv[3] = {0.0, 0.0, 0.0}, t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < DIM; ++q) nv[q] = g[(G_N0 + q) * cap + s];
        if (DIM == 2) {
          t1[0] = -nv[1];
          t1[1] = nv[0];
        } else {
          for (int q = 0; q < 3; ++q) {
            t1[q] = g[(G_T10 + q) * cap + s];
            t2[q] = g[(G_T20 + q) * cap + s];
          }
        }
        const double gdt = g[G_GDT * cap + s], dwn = g[G_DWN * cap + s];
        const double dwt = g[G_DWT * cap + s], kn = g[G_KN * cap + s], kt = g[G_KT * cap + s];
        const double* ri = rin + (int64_t)s * REC;
        double Rold[3] = {ri[0], ri[1], DIM == 3 ? ri[2] : 0.0};
        const int la = ab.x, lb = ab.y;
        double Va[3] = {0, 0, 0}, Wa[3] = {0, 0, 0}, Vb[3] = {0, 0, 0}, Wb[3] = {0, 0, 0};
        for (int k = 0; k < DIM; ++k) Va[k] = sV[k * stride + la];
        for (int k = 0; k < DR; ++k) Wa[k] = sW[k * stride + la];
        const double ra = sr[la];
        double rb = 0.0;
        if (lb >= 0) {
          for (int k = 0; k < DIM; ++k) Vb[k] = sV[k * stride + lb];
          for (int k = 0; k < DR; ++k) Wb[k] = sW[k * stride + lb];
          rb = sr[lb];
        } else {
          const double* u = a.walls_u + (-1 - lb) * DIM;
          for (int k = 0; k < DIM; ++k) Vb[k] = u[k];
        }
        double Rn[3] = {0.0, 0.0, 0.0};
        local_force<DIM>(nv, t1, t2, gdt, dwn, dwt, kn, kt, a.mu, ra, rb, Va, Wa, Vb, Wb, Rold, Rn);
        const double dRn = Rn[0] - Rold[0], dR1 = Rn[1] - Rold[1];
        const double dR2 = DIM == 3 ? Rn[2] - Rold[2] : 0.0;
        double dF[3], dq[3];
        for (int k = 0; k < DIM; ++k) {
          dF[k] = dRn * nv[k] + dR1 * t1[k];
          if (DIM == 3) dF[k] = dF[k] + dR2 * t2[k];
        }
        if (DIM == 2) {
          dq[0] = dR1;
        } else {
          for (int k = 0; k < 3; ++k) dq[k] = dR1 * t2[k] - dR2 * t1[k];
        }
        const double dma = sdm[la], dia = sdi[la];
        for (int k = 0; k < DIM; ++k) sV[k * stride + la] = Va[k] - dma * dF[k];
        for (int k = 0; k < DR; ++k) sW[k * stride + la] = Wa[k] - dia * (ra * dq[k]);
        if (lb >= 0) {
          const double dmb = sdm[lb], dib = sdi[lb];
          for (int k = 0; k < DIM; ++k) sV[k * stride + lb] = Vb[k] + dmb * dF[k];
          for (int k = 0; k < DR; ++k) sW[k * stride + lb] = Wb[k] - dib * (rb * dq[k]);
        }
        // new record: frame force, world force, torque per unit lever
        double* ro = rout + (int64_t)s * REC;
        if (DIM == 2) {
          double4 rec4;
          rec4.x = Rn[0];
          rec4.y = Rn[1];
          rec4.z = Rn[0] * nv[0] + Rn[1] * t1[0];
          rec4.w = Rn[0] * nv[1] + Rn[1] * t1[1];
          *(double4*)ro = rec4;
        } else {
          ro[0] = Rn[0];
          ro[1] = Rn[1];
          ro[2] = Rn[2];
          ro[3] = 0.0;
          for (int k = 0; k < 3; ++k) {
            double fk = Rn[0] * nv[k] + Rn[1] * t1[k];
            ro[4 + k] = fk + Rn[2] * t2[k];
            ro[8 + k] = Rn[1] * t2[k] - Rn[2] * t1[k];
          }
          ro[7] = 0.0;
          ro[11] = 0.0;
        }
        // convergence test values (Sec. 2.1)
        double d2 = 0.0, s2 = 0.0, qq = 0.0;
        for (int k = 0; k < DIM; ++k) {
          double a1 = Rn[k], a0 = Rold[k];
          d2 = d2 + (a1 - a0) * (a1 - a0);
          s2 = s2 + (a1 + a0) * (a1 + a0);
          qq = qq + a1 * a1;
        }
        sumr += sqrt(qq);
        if (d2 < a.alpha * s2 || d2 == 0.0) npass += 1;
        else if (d2 > maxd || d2 != d2) maxd = d2;
      }
      __syncthreads();
    }
  }
  // 3. block reduction (fixed order), partial store, arrival
  for (int off = 32; off > 0; off >>= 1) {
    npass += __shfl_xor(npass, off, 64);
    double o = __shfl_xor(maxd, off, 64);
    if (o > maxd || o != o) maxd = o;
    sumr += __shfl_xor(sumr, off, 64);
  }
  const int wave = tid >> 6, nw = (nthr + 63) >> 6;
  if ((tid & 63) == 0) {
    sh_np[wave] = npass;
    sh_md[wave] = maxd;
    sh_sr[wave] = sumr;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < nw; ++k) {
      npass += sh_np[k];
      if (sh_md[k] > maxd || sh_md[k] != sh_md[k]) maxd = sh_md[k];
      sumr += sh_sr[k];
    }
    BlockPartial* bp = a.partial + b;
    store_rel(&bp->n_pass, npass);
    store_rel((long long*)&bp->max_d_fail, __double_as_longlong(maxd));
    store_rel((long long*)&bp->sum_r, __double_as_longlong(sumr));
    __threadfence();
    unsigned prev = atomicAdd(&st->arrive, 1u);
    sh_last = prev == (unsigned)(a.grid - 1);
  }
  __syncthreads();
  if (!sh_last) return;
  __threadfence();
  // last block: reduce every block's partial in a fixed order and decide
  long long tn = 0;
  double tm = 0.0, ts = 0.0;
  for (int q = tid; q < a.grid; q += nthr) {
    const BlockPartial* bp = a.partial + q;
    tn += load_rel(&bp->n_pass);
    double m = __longlong_as_double(load_rel((const long long*)&bp->max_d_fail));
    if (m > tm || m != m) tm = m;
    ts += __longlong_as_double(load_rel((const long long*)&bp->sum_r));
  }
  for (int off = 32; off > 0; off >>= 1) {
    tn += __shfl_xor(tn, off, 64);
    double o = __shfl_xor(tm, off, 64);
    if (o > tm || o != o) tm = o;
    ts += __shfl_xor(ts, off, 64);
  }
  __syncthreads();
  if ((tid & 63) == 0) {
    sh_np[wave] = tn;
    sh_md[wave] = tm;
    sh_sr[wave] = ts;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < nw; ++k) {
      tn += sh_np[k];
      if (sh_md[k] > tm || sh_md[k] != sh_md[k]) tm = sh_md[k];
      ts += sh_sr[k];
    }
    const long long nc = a.nc;
    const double ravg = ts / (double)nc;
    const double prev = st->r_avg;
    int conv;
    if (a.criterion == 0) {
      conv = (10 * tn >= 9 * nc) && (tn == nc || tm < a.alpha * (prev * prev));
    } else {
      double dd = (ravg - prev) * (ravg - prev);
      double ss = (ravg + prev) * (ravg + prev);
      conv = dd < a.alpha * ss || dd == 0.0;
    }
    st->n_pass = tn;
    st->max_d_fail = tm;
    st->r_avg_prev = prev;
    st->r_avg = ravg;
    st->conv = conv;
    st->iter = j;
    bool finite = isfinite(ts);
    if (!finite) {
      st->done = 1;
      st->status = CD_ENONFINITE;
    } else if (a.fixed_iters > 0) {
      if (j >= a.fixed_iters) {
        st->done = 1;
        st->status = CD_OK;
      }
    } else if (conv) {
      st->done = 1;
      st->status = CD_OK;
    } else if (j >= a.max_iter) {
      st->done = 1;
      st->status = CD_MAXITER;
    }
    st->arrive = 0;
    __threadfence();
  }
}

// R_avg of the starting forces and the solve state (one block, fixed order)
template <int DIM>
__global__ __launch_bounds__(kInitThreads) void k_solve_init(const double* rec0, int64_t nc,
                                                            SolveState* st, int limit) {
  constexpr int REC = DIM == 2 ? 4 : 12;
  __shared__ double sh[kInitThreads / 64];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < nc; q += kInitThreads) {
    const double* rc = rec0 + q * REC;
    double qq = 0.0;
    for (int k = 0; k < DIM; ++k) qq = qq + rc[k] * rc[k];
    s += sqrt(qq);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kInitThreads / 64; ++k) t += sh[k];
    st->iter = 0;
    st->arrive = 0;
    st->n_pass = 0;
    st->max_d_fail = 0.0;
    st->conv = 0;
    st->r_avg = nc > 0 ? t / (double)nc : 0.0;
    st->r_avg_prev = st->r_avg;
    if (nc == 0) {
      st->done = 1;
      st->status = CD_OK;
    } else if (limit <= 0) {
      st->done = 1;
      st->status = CD_MAXITER;
    } else {
      st->done = 0;
      st->status = CD_MAXITER;
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_unslot(const double* rec, const int* contact_slot,
                                               int64_t nc, double* R) {
  constexpr int REC = DIM == 2 ? 4 : 12;
  int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  const double* rc = rec + (int64_t)contact_slot[c] * REC;
  for (int k = 0; k < DIM; ++k) R[k * nc + c] = rc[k];
}

}  // namespace

SweepArgs cd_sweep_args(cd_ctx* c) {
  SweepArgs a;
  a.dom_start = c->dom_start;
  a.dcol = c->dcol;
  a.dncol = c->dncol;
  a.dp = c->dp;
  a.dp_count = c->dp_count;
  a.v = c->v;
  a.w = c->w;
  a.f = c->f;
  a.t = c->t;
  a.r = c->r;
  a.dtim = c->dtim;
  a.dtii = c->dtii;
  a.inc_ptr = c->inc_ptr;
  a.inc = c->inc;
  a.ab = c->slot_ab;
  a.geo = c->geo;
  a.walls_u = c->d_wall + (size_t)c->W * c->dim + c->W;
  a.rec[0] = c->rec[0];
  a.rec[1] = c->rec[1];
  a.state = c->d_state;
  a.partial = c->partial;
  a.P = c->P;
  a.n = (int)c->n;
  a.cap = (int)c->cap;
  a.per_xcd = (c->P + 7) / 8;
  a.grid = 8 * a.per_xcd;
  a.nc = c->nc;
  a.alpha = c->p.alpha;
  a.mu = c->p.mu;
  a.criterion = c->p.criterion;
  a.fixed_iters = c->p.fixed_iters;
  a.max_iter = c->p.max_iter;
  return a;
}

hipError_t cd_launch_solve_init(cd_ctx* c, int limit) {
  if (c->dim == 2)
    hipLaunchKernelGGL(k_solve_init<2>, dim3(1), dim3(kInitThreads), 0, c->stream, c->rec[0], c->nc,
                       c->d_state, limit);
  else
    hipLaunchKernelGGL(k_solve_init<3>, dim3(1), dim3(kInitThreads), 0, c->stream, c->rec[0], c->nc,
                       c->d_state, limit);
  return hipGetLastError();
}

hipError_t cd_launch_sweep(cd_ctx* c) {
  SweepArgs a = cd_sweep_args(c);
  if (c->dim == 2)
    hipLaunchKernelGGL(k_sweep<2>, dim3(a.grid), dim3(c->sweep_threads), c->sweep_lds, c->stream,
                       a);
  else
    hipLaunchKernelGGL(k_sweep<3>, dim3(a.grid), dim3(c->sweep_threads), c->sweep_lds, c->stream,
                       a);
  return hipGetLastError();
}

hipError_t cd_launch_unslot(cd_ctx* c, int final_iter) {
  if (c->nc == 0) return hipSuccess;
  const double* rec = c->rec[final_iter & 1];
  int nb = cd_blocks(c->nc, 256);
  if (c->dim == 2)
    hipLaunchKernelGGL(k_unslot<2>, dim3(nb), dim3(256), 0, c->stream, rec, c->contact_slot, c->nc,
                       c->R);
  else
    hipLaunchKernelGGL(k_unslot<3>, dim3(nb), dim3(256), 0, c->stream, rec, c->contact_slot, c->nc,
                       c->R);
  return hipGetLastError();
}
