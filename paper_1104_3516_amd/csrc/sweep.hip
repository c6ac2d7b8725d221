// sweep.hip - the domain-wise iterative force solve (Sec. 2.1 and 3.1).
//
// One sweep = one launch of k_sweep (one workgroup per domain) followed by
// one launch of k_decide (one workgroup).
//  k_sweep
//   0. Stage the domain's slot data in LDS with coalesced loads: contact
//      frame, force-law constants, the previous sweep's force and the body
//      pair of every native contact.
//   1. Exchange: recompute the velocities of the domain's particles from
//      their base velocities and external forces plus every incident contact
//      force of the previous sweep (native and foreign), into LDS.  This is
//      the per-sweep exchange of boundary contact forces: other domains'
//      forces are read from the previous sweep's record array.
//   2. Sequential update: colours in order; in a colour, lanes update
//      contacts that share no particle, each solving its own force law with
//      all other forces fixed (Eqs. 3-9, Fig. 2) and applying the change to
//      both bodies' LDS velocities.  New forces go to the other record array,
//      so no domain sees a force of the current sweep from another domain
//      (foreign contacts stay frozen for the sweep).
//   3. The workgroup's convergence test values (count passing the relative
//      test, largest change of the others, sum of |R|) go to its partial.
//  k_decide reduces the partials in a fixed order, applies test (I) or (II)
//  and advances the sweep counter; after a stop every later launch of the
//  solve returns at once.
//
// Blocks are mapped to domains so that each of the 8 XCDs (blocks are
// dispatched round-robin over them) works on a contiguous run of domains,
// which are spatial neighbours in the bisection tree and share halo data in
// that XCD's L2.
#include "cd_internal.h"

namespace {

constexpr int kDecideThreads = 1024;

template <int DIM>
struct Layout {
  static constexpr int DR = DIM == 2 ? 1 : 3;
  static constexpr int REC = DIM == 2 ? 4 : 12;
  static constexpr int NG = DIM == 2 ? 2 : 9;      // frame doubles per slot
  static constexpr int PD = DIM + DR + 3;          // staged doubles per particle
  static constexpr int SD = NG + 5 + DIM;          // staged doubles per slot
};

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

template <int DIM, bool GLOB>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
  using L = Layout<DIM>;
  constexpr int DR = L::DR, REC = L::REC, NG = L::NG, PD = L::PD, SD = L::SD;
  extern __shared__ double lds[];
  __shared__ long long sh_np[4];
  __shared__ double sh_md[4], sh_sr[4];

  const SolveState* st = a.state;
  if (*(volatile const int*)&st->done) return;
  const int j = *(volatile const int*)&st->iter + 1;
  const double* rin = a.rec[(j - 1) & 1];
  double* rout = a.rec[j & 1];
  const int b = blockIdx.x;
  const int d = (b % 8) * a.per_xcd + b / 8;
  const int tid = threadIdx.x, nthr = blockDim.x;

  long long npass = 0;
  double maxd = 0.0, sumr = 0.0;

  if (d < a.P) {
    const int cs = a.dom_start[d], nct = a.dom_start[d + 1] - cs;
    const int ps = a.dp_start[d], np = a.dp_start[d + 1] - ps;
    // staging: particles [PD][np], slots [SD][nct], body pairs [nct]
    double* sp = GLOB ? a.gscr + (int64_t)PD * ps : lds;
    double* ss = GLOB ? a.gscr + (int64_t)PD * 2 * a.cap + (int64_t)SD * cs : sp + PD * np;
    int2* sab = GLOB ? (int2*)(a.gscr + (int64_t)PD * 2 * a.cap + (int64_t)SD * a.cap) + cs
                     : (int2*)(ss + SD * nct);
    double* sV = sp;
    double* sW = sV + DIM * np;
    double* sdm = sW + DR * np;
    double* sdi = sdm + np;
    double* sr = sdi + np;
    // 0. stage the native contacts
    const int64_t cap = a.cap;
    const double* g = a.geo;
    for (int k = tid; k < nct; k += nthr) {
      const int s = cs + k;
      for (int q = 0; q < NG; ++q) ss[q * nct + k] = g[q * cap + s];
      for (int q = 0; q < 5; ++q) ss[(NG + q) * nct + k] = g[(G_GDT + q) * cap + s];
      const double* ri = rin + (int64_t)s * REC;
      for (int q = 0; q < DIM; ++q) ss[(NG + 5 + q) * nct + k] = ri[q];
      sab[k] = a.ab[s];
    }
    // 1. exchange: velocities from the previous sweep's forces
    const int64_t E = a.dpe;
    for (int l = tid; l < np; l += nthr) {
      const int64_t e = ps + l;
      double acc[DIM], tacc[DR];
      int q = DIM + DR;
      for (int k = 0; k < DIM; ++k) acc[k] = a.dpb[(q + k) * E + e];
      q += DIM;
      for (int k = 0; k < DR; ++k) tacc[k] = a.dpb[(q + k) * E + e];
      q += DR;
      const double dm = a.dpb[q * E + e], di = a.dpb[(q + 1) * E + e];
      const double rp = a.dpb[(q + 2) * E + e];
      const int e1 = a.dinc_ptr[e + 1];
      for (int x = a.dinc_ptr[e]; x < e1; ++x) {
        const int ent = a.dinc[x];
        const double* rc = rin + (int64_t)(ent >> 1) * REC;
        if (DIM == 2) {
          const double4 r4 = *(const double4*)rc;
          if (ent & 1) {
            acc[0] = acc[0] + r4.z;
            acc[1] = acc[1] + r4.w;
          } else {
            acc[0] = acc[0] - r4.z;
            acc[1] = acc[1] - r4.w;
          }
          tacc[0] = tacc[0] - rp * r4.y;
        } else {
          for (int k = 0; k < 3; ++k) {
            double F = rc[4 + k];
            acc[k] = (ent & 1) ? acc[k] + F : acc[k] - F;
          }
          for (int k = 0; k < 3; ++k) tacc[k] = tacc[k] - rp * rc[8 + k];
        }
      }
      for (int k = 0; k < DIM; ++k) sV[k * np + l] = a.dpb[k * E + e] + dm * acc[k];
      for (int k = 0; k < DR; ++k) sW[k * np + l] = a.dpb[(DIM + k) * E + e] + di * tacc[k];
      sdm[l] = dm;
      sdi[l] = di;
      sr[l] = rp;
    }
    __syncthreads();
    // 2. colour-major sequential update, from the staged data
    const int ncol = a.dncol[d];
    const int* co = a.dcol + (int64_t)d * (CD_MAX_COLORS + 1);
    for (int col = 0; col < ncol; ++col) {
      const int k0 = co[col], k1 = co[col + 1];
      for (int k = k0 + tid; k < k1; k += nthr) {
        const int2 ab = sab[k];
        double nv[3] = {0.0, 0.0, 0.0}, t1[3] = {0.0, 0.0, 0.0}, t2[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < DIM; ++q) nv[q] = ss[q * nct + k];
        if (DIM == 2) {
          t1[0] = -nv[1];
          t1[1] = nv[0];
        } else {
          for (int q = 0; q < 3; ++q) {
            t1[q] = ss[(3 + q) * nct + k];
            t2[q] = ss[(6 + q) * nct + k];
          }
        }
        const double gdt = ss[NG * nct + k], dwn = ss[(NG + 1) * nct + k];
        const double dwt = ss[(NG + 2) * nct + k], kn = ss[(NG + 3) * nct + k];
        const double kt = ss[(NG + 4) * nct + k];
        double Rold[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < DIM; ++q) Rold[q] = ss[(NG + 5 + q) * nct + k];
        const int la = ab.x, lb = ab.y;
        double Va[3] = {0, 0, 0}, Wa[3] = {0, 0, 0}, Vb[3] = {0, 0, 0}, Wb[3] = {0, 0, 0};
        for (int q = 0; q < DIM; ++q) Va[q] = sV[q * np + la];
        for (int q = 0; q < DR; ++q) Wa[q] = sW[q * np + la];
        const double ra = sr[la];
        double rb = 0.0;
        if (lb >= 0) {
          for (int q = 0; q < DIM; ++q) Vb[q] = sV[q * np + lb];
          for (int q = 0; q < DR; ++q) Wb[q] = sW[q * np + lb];
          rb = sr[lb];
        } else {
          const double* u = a.walls_u + (-1 - lb) * DIM;
          for (int q = 0; q < DIM; ++q) Vb[q] = u[q];
        }
        double Rn[3] = {0.0, 0.0, 0.0};
        local_force<DIM>(nv, t1, t2, gdt, dwn, dwt, kn, kt, a.mu, ra, rb, Va, Wa, Vb, Wb, Rold, Rn);
        const double dRn = Rn[0] - Rold[0], dR1 = Rn[1] - Rold[1];
        const double dR2 = DIM == 3 ? Rn[2] - Rold[2] : 0.0;
        double dF[3], dq[3];
        for (int q = 0; q < DIM; ++q) {
          dF[q] = dRn * nv[q] + dR1 * t1[q];
          if (DIM == 3) dF[q] = dF[q] + dR2 * t2[q];
        }
        if (DIM == 2) {
          dq[0] = dR1;
        } else {
          for (int q = 0; q < 3; ++q) dq[q] = dR1 * t2[q] - dR2 * t1[q];
        }
        const double dma = sdm[la], dia = sdi[la];
        for (int q = 0; q < DIM; ++q) sV[q * np + la] = Va[q] - dma * dF[q];
        for (int q = 0; q < DR; ++q) sW[q * np + la] = Wa[q] - dia * (ra * dq[q]);
        if (lb >= 0) {
          const double dmb = sdm[lb], dib = sdi[lb];
          for (int q = 0; q < DIM; ++q) sV[q * np + lb] = Vb[q] + dmb * dF[q];
          for (int q = 0; q < DR; ++q) sW[q * np + lb] = Wb[q] - dib * (rb * dq[q]);
        }
        // new record: frame force, world force, torque per unit lever
        double* ro = rout + (int64_t)(cs + k) * REC;
        if (DIM == 2) {
          double4 rec4;
          rec4.x = Rn[0];
          rec4.y = Rn[1];
          rec4.z = Rn[0] * nv[0] + Rn[1] * t1[0];
          rec4.w = Rn[0] * nv[1] + Rn[1] * t1[1];
          *(double4*)ro = rec4;
        } else {
          double F[3], Q[3];
          for (int q = 0; q < 3; ++q) {
            double fk = Rn[0] * nv[q] + Rn[1] * t1[q];
            F[q] = fk + Rn[2] * t2[q];
            Q[q] = Rn[1] * t2[q] - Rn[2] * t1[q];
          }
          *(double4*)ro = make_double4(Rn[0], Rn[1], Rn[2], 0.0);
          *(double4*)(ro + 4) = make_double4(F[0], F[1], F[2], 0.0);
          *(double4*)(ro + 8) = make_double4(Q[0], Q[1], Q[2], 0.0);
        }
        // convergence test values (Sec. 2.1)
        double d2 = 0.0, s2 = 0.0, qq = 0.0;
        for (int q = 0; q < DIM; ++q) {
          double a1 = Rn[q], a0 = Rold[q];
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
  // 3. block reduction in a fixed order; the partial is read by k_decide
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
    BlockPartial p;
    p.n_pass = npass;
    p.max_d_fail = maxd;
    p.sum_r = sumr;
    p.pad = 0;
    a.partial[b] = p;
  }
}

// stop decision of the sweep just done: one workgroup, fixed reduction order
__global__ __launch_bounds__(kDecideThreads) void k_decide(SweepArgs a) {
  __shared__ long long sh_np[kDecideThreads / 64];
  __shared__ double sh_md[kDecideThreads / 64], sh_sr[kDecideThreads / 64];
  SolveState* st = a.state;
  if (st->done) return;
  const int tid = threadIdx.x;
  long long tn = 0;
  double tm = 0.0, ts = 0.0;
  for (int q = tid; q < a.grid; q += kDecideThreads) {
    const BlockPartial p = a.partial[q];
    tn += p.n_pass;
    if (p.max_d_fail > tm || p.max_d_fail != p.max_d_fail) tm = p.max_d_fail;
    ts += p.sum_r;
  }
  for (int off = 32; off > 0; off >>= 1) {
    tn += __shfl_xor(tn, off, 64);
    double o = __shfl_xor(tm, off, 64);
    if (o > tm || o != o) tm = o;
    ts += __shfl_xor(ts, off, 64);
  }
  const int wave = tid >> 6;
  if ((tid & 63) == 0) {
    sh_np[wave] = tn;
    sh_md[wave] = tm;
    sh_sr[wave] = ts;
  }
  __syncthreads();
  if (tid != 0) return;
  for (int k = 1; k < kDecideThreads / 64; ++k) {
    tn += sh_np[k];
    if (sh_md[k] > tm || sh_md[k] != sh_md[k]) tm = sh_md[k];
    ts += sh_sr[k];
  }
  const long long nc = a.nc;
  const int j = st->iter + 1;
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
  if (!isfinite(ts)) {
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
}

// R_avg of the starting forces and the solve state (one block, fixed order)
template <int DIM>
__global__ __launch_bounds__(kDecideThreads) void k_solve_init(const double* rec0, int64_t nc,
                                                              SolveState* st, int limit) {
  constexpr int REC = DIM == 2 ? 4 : 12;
  __shared__ double sh[kDecideThreads / 64];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < nc; q += kDecideThreads) {
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
    for (int k = 0; k < kDecideThreads / 64; ++k) t += sh[k];
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
  a.dp_start = c->dp_start;
  a.gscr = c->gscr;
  a.dpb = c->dpb;
  a.dpe = 2 * c->cap;
  a.dinc_ptr = c->dinc_ptr;
  a.dinc = c->dinc;
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
    hipLaunchKernelGGL(k_solve_init<2>, dim3(1), dim3(kDecideThreads), 0, c->stream, c->rec[0],
                       c->nc, c->d_state, limit);
  else
    hipLaunchKernelGGL(k_solve_init<3>, dim3(1), dim3(kDecideThreads), 0, c->stream, c->rec[0],
                       c->nc, c->d_state, limit);
  return hipGetLastError();
}

hipError_t cd_launch_sweep(cd_ctx* c, hipEvent_t before, hipEvent_t after) {
  SweepArgs a = cd_sweep_args(c);
  if (before) {
    hipError_t e = hipEventRecord(before, c->stream);
    if (e != hipSuccess) return e;
  }
  dim3 grid(a.grid), block(c->sweep_threads);
  if (c->dim == 2) {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_sweep<2, true>), grid, block, 0, c->stream, a);
    else
      hipLaunchKernelGGL((k_sweep<2, false>), grid, block, c->sweep_lds, c->stream, a);
  } else {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_sweep<3, true>), grid, block, 0, c->stream, a);
    else
      hipLaunchKernelGGL((k_sweep<3, false>), grid, block, c->sweep_lds, c->stream, a);
  }
  if (after) {
    hipError_t e = hipEventRecord(after, c->stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideThreads), 0, c->stream, a);
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
