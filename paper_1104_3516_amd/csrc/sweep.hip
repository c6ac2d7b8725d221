// sweep.hip - the domain-wise iterative force solve (Sec. 2.1 and 3.1).
//
// One wavefront sweeps one domain; a 256-thread workgroup carries four
// domains.  The whole solve of a time step runs in one launch of k_solve
// (a grid barrier after every sweep); k_sweep + k_decide do one sweep per
// launch pair and give the same results.
//  per domain and sweep
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
//   3. The convergence test values (count passing the relative test,
//      largest change of the others, sum of |R|) are reduced per workgroup.
//  The stop decision reduces the workgroup partials in a fixed order and
//  applies test (I) or (II).
//
// Blocks are mapped to domains so that each of the 8 XCDs (blocks are
// dispatched round-robin over them) works on a contiguous run of domains,
// which are spatial neighbours in the bisection tree and share halo data in
// that XCD's L2.
#include "cd_internal.h"

namespace {

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

constexpr int kMaxBlock = 256;

// The domain of block b in pass k.  Block b runs on XCD x = b % 8
// (round-robin dispatch); XCD x owns the contiguous domain range
// [x per, (x+1) per) of the bisection order, so neighbouring domains share
// that XCD's L2.  G8 blocks per XCD.  Returns -1 past the range.
__device__ inline int domain_of(const SweepArgs& a, int b, int k, int G8) {
  const int x = b % 8, i = b / 8;
  const int local = i + k * G8;
  if (local >= a.per_xcd) return -1;
  const int d = x * a.per_xcd + local;
  return d < a.P ? d : -1;
}

// Accumulate the previous sweep's contact forces on one particle entry, in
// ascending contact id: acc -= F (body 1) or += F (body 2), tacc -= r q.
template <int DIM>
__device__ inline void gather_forces(const SweepArgs& a, const double* rin, int64_t e, double rp,
                                     double* acc, double* tacc) {
  constexpr int REC = DIM == 2 ? 4 : 12;
  constexpr int KW = DIM == 2 ? 8 : 16;
  const int* row = a.drow + e * KW;
  if (row[0] == -2) {
    // more incidences than a row holds: the pointer list
    const int e1 = a.dinc_ptr[e + 1];
    for (int x = a.dinc_ptr[e]; x < e1; ++x) {
      const int ent = a.dinc[x];
      const double* rc = rin + (int64_t)(ent >> 1) * REC;
      if (DIM == 2) {
        const double4 r4 = *(const double4*)rc;
        acc[0] = (ent & 1) ? acc[0] + r4.z : acc[0] - r4.z;
        acc[1] = (ent & 1) ? acc[1] + r4.w : acc[1] - r4.w;
        tacc[0] = tacc[0] - rp * r4.y;
      } else {
        for (int k = 0; k < 3; ++k) {
          double F = rc[4 + k];
          acc[k] = (ent & 1) ? acc[k] + F : acc[k] - F;
        }
        for (int k = 0; k < 3; ++k) tacc[k] = tacc[k] - rp * rc[8 + k];
      }
    }
    return;
  }
  // rows hold the valid entries first: gathers in groups of four in flight
  for (int g = 0; g < KW; g += 4) {
    const int4 r4i = *(const int4*)(row + g);
    const int ent[4] = {r4i.x, r4i.y, r4i.z, r4i.w};
    if (ent[0] < 0) break;
    if (DIM == 2) {
      double4 rec[4];
      for (int u = 0; u < 4; ++u)
        if (ent[u] >= 0) rec[u] = *(const double4*)(rin + (int64_t)(ent[u] >> 1) * REC);
      for (int u = 0; u < 4; ++u) {
        if (ent[u] < 0) break;
        acc[0] = (ent[u] & 1) ? acc[0] + rec[u].z : acc[0] - rec[u].z;
        acc[1] = (ent[u] & 1) ? acc[1] + rec[u].w : acc[1] - rec[u].w;
        tacc[0] = tacc[0] - rp * rec[u].y;
      }
    } else {
      double4 fq[4][2];
      for (int u = 0; u < 4; ++u)
        if (ent[u] >= 0) {
          const double* rc = rin + (int64_t)(ent[u] >> 1) * REC;
          fq[u][0] = *(const double4*)(rc + 4);
          fq[u][1] = *(const double4*)(rc + 8);
        }
      for (int u = 0; u < 4; ++u) {
        if (ent[u] < 0) break;
        const double F[3] = {fq[u][0].x, fq[u][0].y, fq[u][0].z};
        const double Q[3] = {fq[u][1].x, fq[u][1].y, fq[u][1].z};
        for (int k = 0; k < 3; ++k) acc[k] = (ent[u] & 1) ? acc[k] + F[k] : acc[k] - F[k];
        for (int k = 0; k < 3; ++k) tacc[k] = tacc[k] - rp * Q[k];
      }
    }
  }
}

// One sweep of domain d by the calling workgroup: stage, exchange, colour-
// major update; accumulates the convergence test values of its contacts.
template <int DIM, bool GLOB>
__device__ inline void sweep_domain(const SweepArgs& a, int d, const double* rin, double* rout,
                                    double* lds, int* s_co, long long& npass, double& maxd,
                                    double& sumr) {
  using L = Layout<DIM>;
  constexpr int DR = L::DR, REC = L::REC, NG = L::NG, PD = L::PD, SD = L::SD;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int* dd = a.ddesc + 8 * (int64_t)d;
  const int cs = dd[0], nct = dd[1], ps = dd[2], np = dd[3], ncol = dd[4];
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
  const int64_t cap = a.cap;
  const double* g = a.geo;
  // 0. colour offsets, and this thread's first native contact (issued
  //    before the particle gathers so that the latencies overlap)
  for (int q = tid; q <= ncol; q += nthr) s_co[q] = a.dcol[(int64_t)d * (CD_MAX_COLORS + 1) + q];
  double sv[SD];
  int2 abv = make_int2(0, 0);
  if (tid < nct) {
    const int s = cs + tid;
    for (int q = 0; q < NG; ++q) sv[q] = g[q * cap + s];
    for (int q = 0; q < 5; ++q) sv[NG + q] = g[(G_GDT + q) * cap + s];
    const double* ri = rin + (int64_t)s * REC;
    for (int q = 0; q < DIM; ++q) sv[NG + 5 + q] = ri[q];
    abv = a.ab[s];
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
    gather_forces<DIM>(a, rin, e, rp, acc, tacc);
    for (int k = 0; k < DIM; ++k) sV[k * np + l] = a.dpb[k * E + e] + dm * acc[k];
    for (int k = 0; k < DR; ++k) sW[k * np + l] = a.dpb[(DIM + k) * E + e] + di * tacc[k];
    sdm[l] = dm;
    sdi[l] = di;
    sr[l] = rp;
  }
  if (tid < nct) {
    for (int q = 0; q < SD; ++q) ss[q * nct + tid] = sv[q];
    sab[tid] = abv;
  }
  for (int k = tid + nthr; k < nct; k += nthr) {
    const int s = cs + k;
    for (int q = 0; q < NG; ++q) ss[q * nct + k] = g[q * cap + s];
    for (int q = 0; q < 5; ++q) ss[(NG + q) * nct + k] = g[(G_GDT + q) * cap + s];
    const double* ri = rin + (int64_t)s * REC;
    for (int q = 0; q < DIM; ++q) ss[(NG + 5 + q) * nct + k] = ri[q];
    sab[k] = a.ab[s];
  }
  __syncthreads();
  // 2. colour-major sequential update, from the staged data
  for (int col = 0; col < ncol; ++col) {
    const int k0 = s_co[col], k1 = s_co[col + 1];
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

struct BlockRed {
  long long np[kMaxBlock / 64];
  double md[kMaxBlock / 64], sr[kMaxBlock / 64];
};

// Fixed-order reduction of per-thread test values over the workgroup;
// thread 0 gets the totals.
__device__ inline BlockPartial block_partial(long long npass, double maxd, double sumr,
                                             BlockRed& sh) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int off = 32; off > 0; off >>= 1) {
    npass += __shfl_xor(npass, off, 64);
    double o = __shfl_xor(maxd, off, 64);
    if (o > maxd || o != o) maxd = o;
    sumr += __shfl_xor(sumr, off, 64);
  }
  const int wave = tid >> 6, nw = (nthr + 63) >> 6;
  __syncthreads();
  if ((tid & 63) == 0) {
    sh.np[wave] = npass;
    sh.md[wave] = maxd;
    sh.sr[wave] = sumr;
  }
  __syncthreads();
  BlockPartial p;
  p.n_pass = 0;
  p.max_d_fail = 0.0;
  p.sum_r = 0.0;
  p.pad = 0;
  if (tid == 0) {
    for (int k = 1; k < nw; ++k) {
      npass += sh.np[k];
      if (sh.md[k] > maxd || sh.md[k] != sh.md[k]) maxd = sh.md[k];
      sumr += sh.sr[k];
    }
    p.n_pass = npass;
    p.max_d_fail = maxd;
    p.sum_r = sumr;
  }
  return p;
}

// Convergence test (I) or (II) of sweep j from its reduced test values
// (Sec. 2.1), and the stop decision.  Runs in one thread.
__device__ inline void decide_sweep(const SweepArgs& a, SolveState* st, int j, long long tn,
                                    double tm, double ts) {
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
  if (st->done) st->stop_at = j;
}

// Fixed-order reduction of `count` workgroup partials by the calling
// workgroup; thread 0 receives the totals.
__device__ inline BlockPartial reduce_partials(const BlockPartial* part, int count, BlockRed& sh) {
  long long tn = 0;
  double tm = 0.0, ts = 0.0;
  for (int q = threadIdx.x; q < count; q += blockDim.x) {
    const BlockPartial p = part[q];
    tn += p.n_pass;
    if (p.max_d_fail > tm || p.max_d_fail != p.max_d_fail) tm = p.max_d_fail;
    ts += p.sum_r;
  }
  return block_partial(tn, tm, ts, sh);
}

// One sweep per launch: block b sweeps domain_of(b, 0).
template <int DIM, bool GLOB>
__global__ __launch_bounds__(kMaxBlock) void k_sweep(SweepArgs a) {
  extern __shared__ double lds[];
  __shared__ BlockRed red;
  __shared__ int s_co[CD_MAX_COLORS + 1];
  const SolveState* st = a.state;
  if (*(volatile const int*)&st->done) return;
  const int j = *(volatile const int*)&st->iter + 1;
  const double* rin = a.rec[(j - 1) & 1];
  double* rout = a.rec[j & 1];
  const int b = blockIdx.x;
  long long npass = 0;
  double maxd = 0.0, sumr = 0.0;
  const int d = domain_of(a, b, 0, gridDim.x / 8);
  if (d >= 0) sweep_domain<DIM, GLOB>(a, d, rin, rout, lds, s_co, npass, maxd, sumr);
  BlockPartial p = block_partial(npass, maxd, sumr, red);
  if (threadIdx.x == 0) a.partial[b] = p;
}

// stop decision of the sweep just done: one workgroup
__global__ __launch_bounds__(1024) void k_decide(SweepArgs a) {
  __shared__ struct {
    long long np[16];
    double md[16], sr[16];
  } red16;
  SolveState* st = a.state;
  if (st->done) return;
  long long tn = 0;
  double tm = 0.0, ts = 0.0;
  for (int q = threadIdx.x; q < a.grid; q += blockDim.x) {
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
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red16.np[wave] = tn;
    red16.md[wave] = tm;
    red16.sr[wave] = ts;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
    tn += red16.np[k];
    if (red16.md[k] > tm || red16.md[k] != red16.md[k]) tm = red16.md[k];
    ts += red16.sr[k];
  }
  decide_sweep(a, st, st->iter + 1, tn, tm, ts);
}

__device__ inline int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_release(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p >= target.  Polls are relaxed loads (an acquire per poll
// would invalidate the XCD's L2 under the workgroups still sweeping); the
// caller issues one acquire fence afterwards.  Gives up, raising the abort
// flag, after spin_limit polls so that every wave reaches the kernel's end.
__device__ inline bool wait_at_least(const int* p, int target, GridBar* bar, long long spin_limit) {
  long long spins = 0;
  while (ld_relaxed(p) < target) {
    if (ld_relaxed(&bar->abort)) return false;
    if (++spins > spin_limit) {
      st_release(&bar->abort, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// The whole force solve of one time step in one launch.  All G blocks are
// resident at once (G is sized from the occupancy of this kernel); block b
// runs the domains domain_of(b, k) of its passes k.
// After sweep j every block arrives at a two-level grid barrier (per XCD,
// then across XCDs); the block completing it opens it and owes the stop
// decision of sweep j, which it takes after arriving at barrier j+1, while
// slower blocks are still sweeping.  Past barrier j+1 every block waits for
// that decision: a stop leaves the forces of sweep j final, since sweep j+1
// wrote the other record array.  Every wait is bounded (abort flag).
template <int DIM, bool GLOB>
__global__ __launch_bounds__(kMaxBlock) void k_solve(SweepArgs a, GridBar* bar, int G, int limit,
                                                    long long spin_limit) {
  extern __shared__ double lds[];
  __shared__ BlockRed red;
  __shared__ int s_co[CD_MAX_COLORS + 1];
  __shared__ int s_last, s_stop;
  SolveState* st = a.state;
  if (*(volatile const int*)&st->done) return;   // nothing to solve: every block returns
  const int b = blockIdx.x, x = b % 8, G8 = G / 8;
  int owe = 0;   // sweep whose decision this block owes (0: none)
  auto decide = [&](int jd) {
    BlockPartial t = reduce_partials(a.partial + (int64_t)(jd & 1) * G, G, red);
    if (threadIdx.x == 0) {
      if (!__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        decide_sweep(a, st, jd, t.n_pass, t.max_d_fail, t.sum_r);
      st_release(&bar->dec, jd);
    }
  };
  for (int j = 1; j <= limit; ++j) {
    const double* rin = a.rec[(j - 1) & 1];
    double* rout = a.rec[j & 1];
    long long npass = 0;
    double maxd = 0.0, sumr = 0.0;
    for (int k = 0;; ++k) {
      const int d = domain_of(a, b, k, G8);
      if (d < 0) break;
      sweep_domain<DIM, GLOB>(a, d, rin, rout, lds, s_co, npass, maxd, sumr);
    }
    BlockPartial p = block_partial(npass, maxd, sumr, red);
    if (threadIdx.x == 0) {
      a.partial[(int64_t)(j & 1) * G + b] = p;
      // this block's forces and partial, device-wide, before the arrival
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      int last = 0;
      unsigned prev = __hip_atomic_fetch_add(&bar->xcount[x][j & 1], 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      if (prev == (unsigned)(G8 - 1)) {
        // last of this XCD: pass the arrivals on
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(&bar->xcount[x][j & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned prev2 = __hip_atomic_fetch_add(&bar->count[j & 1], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        if (prev2 == 7u) {
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
          __hip_atomic_store(&bar->count[j & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          st_release(&bar->gen, j);   // barrier j is open
          last = 1;
        }
      }
      s_last = last;
    }
    __syncthreads();
    // the decision this block owes for sweep j-1 (its partials are in the
    // other buffer, untouched until every block has seen that decision)
    if (owe) {
      decide(owe);
      owe = 0;
    }
    if (s_last) owe = j;
    if (threadIdx.x == 0) {
      bool ok = wait_at_least(&bar->gen, j, bar, spin_limit);
      ok = ok && wait_at_least(&bar->dec, j - 1, bar, spin_limit);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      // only a stop decided for a sweep before j counts here: the decision
      // of sweep j may already be out while this block is still at barrier j
      const int stop = __hip_atomic_load(&st->stop_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_stop = !ok || (stop != 0 && stop <= j - 1);
    }
    __syncthreads();
    if (s_stop) break;
  }
  // the decision of the last sweep (at the sweep limit)
  if (owe) decide(owe);
}

// R_avg of the starting forces and the solve state (one block, fixed order)
template <int DIM>
__global__ __launch_bounds__(1024) void k_solve_init(const double* rec0, int64_t nc,
                                                    SolveState* st, int limit, GridBar* bar) {
  constexpr int REC = DIM == 2 ? 4 : 12;
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < nc; q += blockDim.x) {
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
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    for (int x = 0; x < 8; ++x) bar->xcount[x][0] = bar->xcount[x][1] = 0;
    bar->count[0] = bar->count[1] = 0;
    bar->gen = 0;
    bar->dec = 0;
    bar->abort = 0;
    st->iter = 0;
    st->arrive = 0;
    st->n_pass = 0;
    st->max_d_fail = 0.0;
    st->conv = 0;
    st->r_avg = nc > 0 ? t / (double)nc : 0.0;
    st->r_avg_prev = st->r_avg;
    st->stop_at = 0;
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
  a.drow = c->drow;
  a.ddesc = c->ddesc;
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
    hipLaunchKernelGGL(k_solve_init<2>, dim3(1), dim3(1024), 0, c->stream, c->rec[0], c->nc,
                       c->d_state, limit, c->d_bar);
  else
    hipLaunchKernelGGL(k_solve_init<3>, dim3(1), dim3(1024), 0, c->stream, c->rec[0], c->nc,
                       c->d_state, limit, c->d_bar);
  return hipGetLastError();
}

static size_t block_lds(cd_ctx* c) { return c->sweep_global ? 0 : c->sweep_lds; }

hipError_t cd_launch_sweep(cd_ctx* c, hipEvent_t before, hipEvent_t after) {
  SweepArgs a = cd_sweep_args(c);
  if (before) {
    hipError_t e = hipEventRecord(before, c->stream);
    if (e != hipSuccess) return e;
  }
  dim3 grid(a.grid), block(c->sweep_block);
  if (c->dim == 2) {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_sweep<2, true>), grid, block, 0, c->stream, a);
    else
      hipLaunchKernelGGL((k_sweep<2, false>), grid, block, block_lds(c), c->stream, a);
  } else {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_sweep<3, true>), grid, block, 0, c->stream, a);
    else
      hipLaunchKernelGGL((k_sweep<3, false>), grid, block, block_lds(c), c->stream, a);
  }
  if (after) {
    hipError_t e = hipEventRecord(after, c->stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(1024), 0, c->stream, a);
  return hipGetLastError();
}

template <int DIM, bool GLOB>
static int solve_capacity(cd_ctx* c) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve<DIM, GLOB>, c->sweep_block,
                                                   block_lds(c)) != hipSuccess)
    return 0;
  return per_cu * c->num_cu;
}

int cd_solve_grid(cd_ctx* c) {
  int cap;
  if (c->dim == 2) cap = c->sweep_global ? solve_capacity<2, true>(c) : solve_capacity<2, false>(c);
  else cap = c->sweep_global ? solve_capacity<3, true>(c) : solve_capacity<3, false>(c);
  const int want = cd_sweep_args(c).grid;
  int g = want < cap ? want : cap;
  return (g / 8) * 8;
}

hipError_t cd_launch_solve(cd_ctx* c, int G, int limit) {
  SweepArgs a = cd_sweep_args(c);
  const long long spin_limit = 1ll << 26;
  dim3 grid(G), block(c->sweep_block);
  if (c->dim == 2) {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_solve<2, true>), grid, block, 0, c->stream, a, c->d_bar, G, limit,
                         spin_limit);
    else
      hipLaunchKernelGGL((k_solve<2, false>), grid, block, block_lds(c), c->stream, a, c->d_bar, G,
                         limit, spin_limit);
  } else {
    if (c->sweep_global)
      hipLaunchKernelGGL((k_solve<3, true>), grid, block, 0, c->stream, a, c->d_bar, G, limit,
                         spin_limit);
    else
      hipLaunchKernelGGL((k_solve<3, false>), grid, block, block_lds(c), c->stream, a, c->d_bar, G,
                         limit, spin_limit);
  }
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
